#!/usr/bin/env python3
"""Throughput of the MI355X harmonic sum on the 1D DM-trial batch.

Workload (default): 1000 spectra x 2^21 FP32 bins of exponential (chi-square,
2 dof, mean 1) noise, 1% of them carrying a harmonic comb at a random
fractional fundamental (16 harmonics, amplitude 5/sqrt(i)); Hmax = 32; outputs
h for H = 1, 2, 4, 8, 16, 32 plus per-bin max-SNR and best-H.

One step = one pass of the whole 1D hot path over the batch, inputs already
resident in HBM: FP64 statistics + SNR constants, then the harmonic sum of each
of the four variants (eq. (1) standard, Max, freq-bin, Greedy; arXiv:1812.02647
eq. (1)-(4)). value = input bins of the batch / step time.

Prints one JSON line. Extra objects:
  roofline      -- the dominant kernel (the variant with the longest launch):
                   algorithmic bytes per launch / its mean launch time (HIP
                   events on the launch stream) against the 8 TB/s HBM peak;
  cpu_baseline  -- the CPU oracle (as it stands) on a bounded sample of the
                   same batch, one spectrum per thread on the host cores;
  per_variant   -- every variant's launch time, G bins/s and HBM fraction.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G input bins/s and % of HBM peak, 1D batch Hmax=32, FP32 vs FP16-storage"
HBM_PEAK_GBS = 8000.0
VARIANT_NAMES = ["eq1", "max", "freqbin", "greedy"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-spectra", type=int, default=1000)
    ap.add_argument("--n-bins", type=int, default=1 << 21)
    ap.add_argument("--hmax", type=int, default=32)
    ap.add_argument("--variants", default="eq1,max,freqbin,greedy")
    ap.add_argument("--cpu-baseline-spectra", type=int, default=96,
                    help="spectra in the oracle's timed sample (0 skips it)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: min(16, cores)")
    return ap.parse_args()


def alg_bytes_per_launch(variant: int, total_bins: int, h_floats: int, in_bytes: int) -> int:
    """Compulsory HBM bytes of one harmonic-sum launch over the batch: each
    input bin read once, each output written once (h planes, max-SNR, best-H)."""
    return total_bins * in_bytes + 4 * h_floats + 4 * total_bins + 1 * total_bins


def cpu_baseline(x, offsets, hmax, variants, n_sample, threads):
    """The oracle on n_sample spectra of the batch: statistics and every
    variant of each spectrum, one spectrum per task on a thread pool (ctypes
    releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    O.lib()
    picks = np.linspace(0, offsets.size - 2, n_sample).astype(int)

    def work(s):
        xs = x[offsets[s]:offsets[s + 1]].astype(np.float64)
        mu, sd = O.stats(xs)
        for v in variants:
            O.hrms_1d(xs, v, hmax, f32=True, mu=mu, sigma=sd)
        return xs.size

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        bins = sum(ex.map(work, picks))
    dt = time.perf_counter() - t0
    return {"value": bins / dt / 1e9, "unit": "G input bins/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sample} of the batch's spectra x {offsets[1] - offsets[0]} bins, "
                      f"statistics + {len(variants)} variants each, FP32 evaluation, "
                      f"{dt:.1f} s wall on {threads} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the harmonic sum of "
              "independent spectra shards by spectrum with no exchange, which this "
              "single-GPU build does not launch.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1812_02647_amd import hrms as H
    from paper_1812_02647_amd import synth

    variants = [VARIANT_NAMES.index(v) for v in args.variants.split(",")]
    ns, nb, hmax = args.n_spectra, args.n_bins, args.hmax

    t0 = time.perf_counter()
    x, offsets, combs = synth.batch(ns, nb, seed=synth.SEED_BASE + 1)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    xd = torch.from_numpy(x).to(dev)
    total = int(offsets[-1])

    handle = H.hrms_create(0)
    stream = torch.cuda.current_stream()
    stats = torch.zeros((ns, 2), dtype=torch.float64, device=dev)
    # shared output buffers, sized for the largest layout (eq. (1): N floats per level)
    layouts = {}
    for v in variants:
        b = H.hrms_run1d_args()
        b.n_spectra, b.variant, b.dtype, b.hmax_all = ns, v, H.HRMS_F32, hmax
        b.offsets = offsets.ctypes.data
        layouts[v] = H.hrms_layout_1d(b)[1]
    h_buf = torch.empty(max(layouts.values()), dtype=torch.float32, device=dev)
    ms_buf = torch.empty(total, dtype=torch.float32, device=dev)
    bh_buf = torch.empty(total, dtype=torch.uint8, device=dev)

    def make_args(v, mode, mask):
        a = H.hrms_run1d_args()
        a.n_spectra, a.variant, a.dtype, a.hmax_all = ns, v, H.HRMS_F32, hmax
        a.out_mask, a.stats_mode = mask, mode
        a.x, a.offsets = xd.data_ptr(), offsets.ctypes.data
        a.stats = stats.data_ptr()
        a.h, a.max_snr, a.best_h = h_buf.data_ptr(), ms_buf.data_ptr(), bh_buf.data_ptr()
        return a

    stats_args = make_args(variants[0], H.HRMS_STATS_COMPUTE, 0)
    run_args = {v: make_args(v, H.HRMS_STATS_PROVIDED, H.HRMS_OUT_ALL) for v in variants}

    def step(events=None):
        if events is not None:
            events[0].record(stream)
        H.hrms_run_1d(handle, stats_args, stream)
        if events is not None:
            events[1].record(stream)
        for k, v in enumerate(variants):
            H.hrms_run_1d(handle, run_args[v], stream)
            if events is not None:
                events[2 + k].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2 + len(variants))]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    tw0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0

    step_ms = [e[0].elapsed_time(e[-1]) for e in ev]
    stats_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    per_variant = {}
    for k, v in enumerate(variants):
        t = float(np.mean([e[1 + k].elapsed_time(e[2 + k]) for e in ev]))
        byts = alg_bytes_per_launch(v, total, layouts[v], 4)
        per_variant[VARIANT_NAMES[v]] = {
            "ms": round(t, 4),
            "gbins_per_s": round(total / (t * 1e-3) / 1e9, 2),
            "alg_bytes": byts,
            "achieved_gbs": round(byts / (t * 1e-3) / 1e9, 1),
            "frac_hbm": round(byts / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        }
    ms_per_step = float(np.mean(step_ms))
    dom = max(per_variant, key=lambda k: per_variant[k]["ms"])
    d = per_variant[dom]

    cpu = None
    if args.cpu_baseline_spectra > 0:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(x, offsets, hmax, variants, args.cpu_baseline_spectra, threads)

    out = {
        "metric": METRIC,
        "value": round(total / (ms_per_step * 1e-3) / 1e9, 3),
        "unit": "G input bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"1D batch: {ns} spectra x {nb} FP32 bins, exponential noise, "
                        f"{len(combs)} fractional combs; Hmax={hmax}; step = FP64 stats + "
                        f"{'+'.join(VARIANT_NAMES[v] for v in variants)}, all outputs",
            "n_spectra": ns, "n_bins": nb, "hmax": hmax,
            "variants": [VARIANT_NAMES[v] for v in variants],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_hrms1d ({dom})",
            "achieved": d["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": d["frac_hbm"],
            "traffic": None,
        },
        "cpu_baseline": cpu,
        "per_variant": per_variant,
        "stats_ms": round(stats_ms, 4),
        "wall_s_timed": round(wall, 3),
        "gen_s": round(t_gen, 1),
    }
    H.hrms_destroy(handle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
