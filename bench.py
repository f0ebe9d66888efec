#!/usr/bin/env python3
"""Throughput of the MI355X harmonic sum (arXiv:1812.02647, eq. (1)-(4)).

Default workload -- the 1D DM-trial batch: 1000 spectra x 2^21 FP32 bins of
exponential (chi-square, 2 dof, mean 1) noise, 1% of them carrying a harmonic
comb at a random fractional fundamental (16 harmonics, amplitude 5/sqrt(i));
Hmax = 32; outputs h for H = 1, 2, 4, 8, 16, 32 plus per-bin max-SNR and
best-H.

One step = one pass of the whole 1D hot path over the batch, inputs already
resident in HBM: FP64 statistics + SNR constants, then the harmonic sum of each
of the four variants (standard eq. (1), Max, freq-bin, Greedy). value = input
bins of the batch / step time.

The JSON line also carries:
  roofline      -- the dominant kernel (the longest launch: a variant's time
                   over its number of harmonic-sum launches, which
                   hrms_plan_1d gives): algorithmic bytes per launch / its
                   mean launch time (HIP events on the launch stream) against
                   the 8 TB/s HBM peak;
  cpu_baseline  -- the CPU oracle (as it stands) on a bounded sample of the
                   same batch, one spectrum per thread on the host cores;
  per_variant   -- every variant's launch time, G bins/s and HBM fraction;
  fp16_storage  -- the same step on the batch normalised to unit mean and
                   stored as FP16 (normalisation timed apart), its speedup over
                   the FP32 step and over plain per-spectrum FP32 launches, and
                   the largest relative difference of its sums from FP32
                   storage (the error against the binary64 oracle is bounded
                   in the test suite).

--workload uneven: 512 spectra of log-uniform length 2^14..2^23 with Hmax in
{8, 16, 32}: one graph-captured persistent launch vs per-spectrum launches.
--workload plane: 85 fdot rows x 2^21 bins, Hmax = 16, all four variants and
Greedy with fdot drift, FP32 and FP16 storage.
The default workload also runs the other two and reports them under "plane"
and "uneven" (--no-sub skips them).
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
# kernels of the default launch shapes
KERNEL_OF = {"eq1": "k_hrms1d_eq1", "max": "k_hrms1d_win", "freqbin": "k_hrms1d_gather",
             "greedy": "k_hrms1d_gather"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch", choices=["batch", "uneven", "plane"])
    ap.add_argument("--n-spectra", type=int, default=1000)
    ap.add_argument("--n-bins", type=int, default=1 << 21)
    ap.add_argument("--hmax", type=int, default=32)
    ap.add_argument("--variants", default="eq1,max,freqbin,greedy")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage form")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the candidate, peak and exhaustive-path timings (only the step's "
                         "launches run, e.g. for a kernel trace whose means match per_variant)")
    ap.add_argument("--cpu-baseline-spectra", type=int, default=400,
                    help="spectra in the oracle's timed sample (0 skips it)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: min(16, cores)")
    ap.add_argument("--no-sub", action="store_true",
                    help="with the default workload, skip the plane and uneven-batch sub-results")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy the input once (a dispatch of known bytes for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


# the kernels and the host planner (tile order, launch shapes) both decide the traffic
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1812_02647_amd", "csrc", f)
                  for f in ("hrms_kernels.hip", "hrms_abi.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(workload: str, variant: str, dtype: str = "f32"):
    """HBM bytes (read + written) per launch of a variant's kernels on a
    workload, from the committed counter runs (FETCH_SIZE, WRITE_SIZE, each
    scaled by what the counter reads for a copy of known size), or None if
    they were taken on other kernel sources."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    digest = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()
    if rec.get("source_sha256") != digest:
        return None
    for ent in rec.get("entries", []):
        if (ent.get("workload"), ent.get("variant"), ent.get("dtype")) == (workload, variant, dtype):
            return ent["read_bytes"] + ent["write_bytes"]
    return None


def alg_bytes_per_pass(total_bins: int, h_floats: int, in_bytes: int) -> int:
    """Compulsory HBM bytes of one variant's harmonic sum over a batch (all its
    launches): each input bin read once, each output written once (h planes,
    max-SNR, best-H). Per launch of a split variant: the same rate, as bytes
    and time both divide by its launches."""
    return total_bins * in_bytes + 4 * h_floats + 4 * total_bins + 1 * total_bins


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, offsets, hmax, variants, n_sample, threads):
    """The oracle on n_sample spectra of the batch: statistics and every
    variant of each spectrum, one spectrum per task on a thread pool (ctypes
    releases the GIL), as the paper parallelises its CPU code over time
    series; plus the same on one thread for a few spectra."""
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
    one = picks[:max(1, min(4, n_sample // threads))]
    t1 = time.perf_counter()
    bins1 = sum(work(s) for s in one)
    dt1 = time.perf_counter() - t1
    return {"value": bins / dt / 1e9, "unit": "G input bins/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sample} of the batch's spectra x {offsets[1] - offsets[0]} bins, "
                      f"statistics + {len(variants)} variants each, FP32 evaluation, "
                      f"{dt:.1f} s wall on {threads} threads",
            "one_thread": {"value": bins1 / dt1 / 1e9, "spectra": len(one)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


class Runner:
    """Batched step over one device batch: statistics pass, then every variant
    (statistics provided), each bracketed by HIP events on the launch stream."""

    def __init__(self, H, handle, xd, offsets, hmax, variants, dtype_code):
        import torch
        self.H, self.handle, self.xd, self.offsets = H, handle, xd, offsets
        self.hmax, self.variants = hmax, variants
        ns = offsets.size - 1
        total = int(offsets[-1])
        dev = xd.device
        self.total = total
        self.stats = torch.zeros((ns, 2), dtype=torch.float64, device=dev)
        self.layouts = {}
        for v in variants:
            b = H.hrms_run1d_args()
            b.n_spectra, b.variant, b.dtype, b.hmax_all = ns, v, dtype_code, hmax
            b.offsets = offsets.ctypes.data
            self.layouts[v] = H.hrms_layout_1d(b)[1]
        self.h = torch.empty(max(self.layouts.values()), dtype=torch.float32, device=dev)
        self.ms = torch.empty(total, dtype=torch.float32, device=dev)
        self.bh = torch.empty(total, dtype=torch.uint8, device=dev)
        self.in_bytes = xd.element_size()
        # the counter records are of the 1000 x 2^21, Hmax = 32 batch
        self.default_batch = (ns == 1000 and total == 1000 * (1 << 21) and hmax == 32)

        def make(v, mode, mask):
            a = H.hrms_run1d_args()
            a.n_spectra, a.variant, a.dtype, a.hmax_all = ns, v, dtype_code, hmax
            a.out_mask, a.stats_mode = mask, mode
            a.x, a.offsets = xd.data_ptr(), offsets.ctypes.data
            a.stats = self.stats.data_ptr()
            a.h, a.max_snr, a.best_h = self.h.data_ptr(), self.ms.data_ptr(), self.bh.data_ptr()
            return a

        self.stats_args = make(variants[0], H.HRMS_STATS_COMPUTE, 0)
        self.run_args = {v: make(v, H.HRMS_STATS_PROVIDED, H.HRMS_OUT_ALL) for v in variants}

    def step(self, stream, events=None):
        H = self.H
        if events is not None:
            events[0].record(stream)
        H.hrms_run_1d(self.handle, self.stats_args, stream)
        if events is not None:
            events[1].record(stream)
        for k, v in enumerate(self.variants):
            H.hrms_run_1d(self.handle, self.run_args[v], stream)
            if events is not None:
                events[2 + k].record(stream)

    def measure(self, steps, warmup):
        import torch
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            self.step(stream)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2 + len(self.variants))]
              for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(stream, ev[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        step_ms = float(np.mean([e[0].elapsed_time(e[-1]) for e in ev]))
        stats_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        per = {}
        for k, v in enumerate(self.variants):
            t = float(np.mean([e[1 + k].elapsed_time(e[2 + k]) for e in ev]))
            byts = alg_bytes_per_pass(self.total, self.layouts[v], self.in_bytes)
            name = VARIANT_NAMES[v]
            shape, launches = self.H.hrms_plan_1d(self.handle, self.run_args[v])
            per[name] = {
                "ms": round(t, 4),
                "launches": launches,
                "mean_launch_ms": round(t / max(1, launches), 4),
                "shape": list(shape),
                "gbins_per_s": round(self.total / (t * 1e-3) / 1e9, 2),
                "alg_bytes": byts,
                "achieved_gbs": round(byts / (t * 1e-3) / 1e9, 1),
                "frac_hbm": round(byts / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": (measured_traffic("batch", name, "f32" if self.in_bytes == 4 else "f16")
                            if self.default_batch else None),
            }
        return step_ms, stats_ms, per, wall


def copy_ceiling(xd) -> float:
    """Measured copy rate (GB/s, bytes read + written) of the input on this
    GPU: the practical ceiling a streaming kernel meets."""
    import torch
    y = torch.empty_like(xd)
    y.copy_(xd)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        y.copy_(xd)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    del y
    return 2.0 * xd.numel() * xd.element_size() / (ms * 1e-3) / 1e9


def per_spectrum_step_ms(H, xd, offsets, hmax, variants):
    """One step as plain per-spectrum launches (statistics computed by each
    launch, no graph capture): the unbatched FP32 form."""
    import torch
    old = os.environ.get("HRMS_NO_GRAPH")
    os.environ["HRMS_NO_GRAPH"] = "1"
    try:
        h = H.hrms_create(0)
    finally:
        if old is None:
            os.environ.pop("HRMS_NO_GRAPH")
        else:
            os.environ["HRMS_NO_GRAPH"] = old
    ns = offsets.size - 1
    n_max = int(np.max(np.diff(offsets)))
    dev = xd.device
    st = torch.zeros(2, dtype=torch.float64, device=dev)
    hb = torch.empty(6 * n_max, dtype=torch.float32, device=dev)
    ms = torch.empty(n_max, dtype=torch.float32, device=dev)
    bh = torch.empty(n_max, dtype=torch.uint8, device=dev)
    args = []
    offs_keep = []
    for s in range(ns):
        for v in variants:
            a = H.hrms_run1d_args()
            o = np.array([0, offsets[s + 1] - offsets[s]], np.int64)
            offs_keep.append(o)
            a.n_spectra, a.variant, a.dtype, a.hmax_all = 1, v, H.HRMS_F32, hmax
            a.out_mask, a.stats_mode = H.HRMS_OUT_ALL, H.HRMS_STATS_COMPUTE
            a.x = xd.data_ptr() + int(offsets[s]) * xd.element_size()
            a.offsets = o.ctypes.data
            a.stats, a.h, a.max_snr, a.best_h = st.data_ptr(), hb.data_ptr(), ms.data_ptr(), bh.data_ptr()
            args.append(a)
    stream = torch.cuda.current_stream()
    for a in args[:len(variants) * 2]:
        H.hrms_run_1d(h, a, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for a in args:
        H.hrms_run_1d(h, a, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    H.hrms_destroy(h)
    return e0.elapsed_time(e1)


def storage_diff(H, handle, xd, offsets, hmax, variants, n_sub):
    """Difference of the h planes computed from FP16 storage against FP32
    storage of the same normalised values x * fl32(1/mu), on the first n_sub
    spectra of the batch: the largest absolute difference, and the largest
    relative difference over sums in FP16's normal range (bins below 2^-14
    lose relative precision in FP16 by construction)."""
    import torch
    sub = np.ascontiguousarray(offsets[:n_sub + 1])
    xs = xd[:int(sub[-1])]
    q = H.hrms_quantize_args()
    st = torch.zeros((n_sub, 2), dtype=torch.float64, device=xd.device)
    so = torch.zeros((n_sub, 2), dtype=torch.float64, device=xd.device)
    y = torch.empty(xs.numel(), dtype=torch.float16, device=xd.device)
    q.n_spectra, q.dtype, q.stats_mode = n_sub, H.HRMS_F16, H.HRMS_STATS_COMPUTE
    q.x, q.offsets, q.stats, q.stats_out, q.y = (xs.data_ptr(), sub.ctypes.data, st.data_ptr(),
                                                 so.data_ptr(), y.data_ptr())
    H.hrms_quantize(handle, q)
    torch.cuda.synchronize()
    inv = (1.0 / st[:, 0]).to(torch.float32)
    xn = xs * torch.repeat_interleave(inv, torch.from_numpy(np.diff(sub)).to(xd.device))
    out = {}
    for v in variants:
        b32 = H.Batch1D(xn, sub, v, hmax, out_mask=H.HRMS_OUT_H).run(handle)
        b16 = H.Batch1D(y, sub, v, hmax, out_mask=H.HRMS_OUT_H).run(handle)
        torch.cuda.synchronize()
        n = b32.h_total
        ref, got = b32.h[:n], b16.h[:n]
        err = (got - ref).abs()
        normal = ref.abs() >= 2.0 ** -14          # FP16's normal range
        # candidate lists at SNR >= 6 from the two storage forms
        lists = []
        for xx, sto in ((xn, so), (y, so)):
            c = H.Batch1D(xx, sub, v, hmax, out_mask=H.HRMS_OUT_CAND, stats=sto.clone(),
                          want_consts=False, cand_capacity=1 << 20, cand_threshold=6.0)
            c.run(handle)
            torch.cuda.synchronize()
            _, rec = c.candidates()
            lists.append({(int(r["spectrum"]), int(r["bin"])): int(r["best_h"]) for r in rec})
        a32, a16 = lists
        both = set(a32) & set(a16)
        out[VARIANT_NAMES[v]] = {
            "max_abs": float(f"{float(err.max()):.3g}"),
            "max_rel_fp16_normal": float(f"{float((err[normal] / ref[normal].abs()).max()):.3g}"),
            "cand_snr6_fp32": len(a32), "cand_snr6_fp16": len(a16),
            "cand_jaccard": round(len(both) / max(1, len(set(a32) | set(a16))), 4),
            "cand_best_h_agree": round(sum(a32[k] == a16[k] for k in both) / max(1, len(both)), 4),
        }
    return out


def extras(args, H, handle, xd, offsets, hmax, variants, total):
    """Candidate list, peak list and exhaustive-path timings on the batch."""
    import torch
    cand = {}
    sa = H.Batch1D(xd, offsets, variants[0], hmax, out_mask=0, want_consts=False).run(handle)
    stc = sa.stats   # statistics computed once, provided to every candidate run
    for v in variants:
        b = H.Batch1D(xd, offsets, v, hmax, out_mask=H.HRMS_OUT_CAND, stats=stc,
                      want_consts=False, cand_capacity=1 << 23, cand_threshold=6.0)
        b.run(handle)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(max(1, args.steps)):
            b.run(handle)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / max(1, args.steps)
        cand[VARIANT_NAMES[v]] = {"ms": round(t, 4), "gbins_per_s": round(total / t / 1e6, 2),
                                  "candidates": b.candidates()[0]}
        del b
        # local maxima only (max-SNR written, then the peak pass over it)
        b = H.Batch1D(xd, offsets, v, hmax, out_mask=H.HRMS_OUT_PEAKS | H.HRMS_OUT_MAXSNR,
                      stats=stc, want_consts=False, cand_capacity=1 << 23, cand_threshold=6.0)
        b.run(handle)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(max(1, args.steps)):
            b.run(handle)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / max(1, args.steps)
        cand[VARIANT_NAMES[v]]["peaks_ms"] = round(t, 4)
        cand[VARIANT_NAMES[v]]["peaks"] = b.candidates()[0]
        del b
    del sa

    # exhaustive-path sum (h only; not part of the step, which holds the
    # paper's four variants)
    ob = H.Batch1D(xd, offsets, H.HRMS_OPT, hmax, out_mask=H.HRMS_OUT_H, stats=stc,
                   want_consts=False)
    ob.run(handle)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(max(1, args.steps)):
        ob.run(handle)
    e1.record()
    torch.cuda.synchronize()
    t_opt = e0.elapsed_time(e1) / max(1, args.steps)
    opt = {"ms": round(t_opt, 4), "gbins_per_s": round(total / t_opt / 1e6, 2),
           "outputs": "h only", "kernel": "k_hrms1d_win (exhaustive path)"}
    del ob, stc
    torch.cuda.empty_cache()

    return cand, opt


def workload_batch(args):
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

    r32 = Runner(H, handle, xd, offsets, hmax, variants, H.HRMS_F32)
    ms_per_step, stats_ms, per_variant, wall = r32.measure(args.steps, args.warmup)
    copy_gbs = copy_ceiling(xd)
    for v in per_variant.values():
        v["frac_copy"] = round(v["achieved_gbs"] / copy_gbs, 4)
    dom = max(per_variant, key=lambda k: per_variant[k]["mean_launch_ms"])
    d = per_variant[dom]
    del r32
    torch.cuda.empty_cache()

    # candidate list, peak list and exhaustive path, outside the step
    cand = {}
    opt = None
    if not args.no_extras:
        cand, opt = extras(args, H, handle, xd, offsets, hmax, variants, total)

    fp16 = None
    if not args.no_fp16:
        y = torch.empty(total, dtype=torch.float16, device=dev)
        qa = H.hrms_quantize_args()
        qa.n_spectra, qa.dtype, qa.stats_mode = ns, H.HRMS_F16, H.HRMS_STATS_COMPUTE
        st_raw = torch.zeros((ns, 2), dtype=torch.float64, device=dev)
        st_out = torch.zeros((ns, 2), dtype=torch.float64, device=dev)
        qa.x, qa.offsets, qa.stats, qa.stats_out, qa.y = (xd.data_ptr(), offsets.ctypes.data,
                                                           st_raw.data_ptr(), st_out.data_ptr(),
                                                           y.data_ptr())
        stream = torch.cuda.current_stream()
        H.hrms_quantize(handle, qa, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        H.hrms_quantize(handle, qa, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        q_ms = e0.elapsed_time(e1)
        r16 = Runner(H, handle, y, offsets, hmax, variants, H.HRMS_F16)
        ms16, stats16, per16, _ = r16.measure(args.steps, args.warmup)
        del r16
        torch.cuda.empty_cache()
        diff = storage_diff(H, handle, xd, offsets, hmax, variants, n_sub=8)
        per_spec_ms = per_spectrum_step_ms(H, xd, offsets, hmax, variants)
        fp16 = {
            "value": round(total / (ms16 * 1e-3) / 1e9, 3),
            "unit": "G input bins/s",
            "ms_per_step": round(ms16, 4),
            "normalise_quantise_ms": round(q_ms, 4),
            "per_variant": per16,
            "speedup_vs_fp32_batched": round(ms_per_step / ms16, 3),
            "fp32_per_spectrum_ms_per_step": round(per_spec_ms, 3),
            "speedup_vs_fp32_per_spectrum": round(per_spec_ms / ms16, 3),
            "diff_vs_fp32_storage": diff,
        }

    if args.calibrate_copy:
        y = torch.empty_like(xd)
        y.copy_(xd)
        torch.cuda.synchronize()
        del y

    cpu = None
    if args.cpu_baseline_spectra > 0:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(x, offsets, hmax, variants, min(args.cpu_baseline_spectra, ns),
                           threads)
    H.hrms_destroy(handle)
    return {
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
            "kernel": f"{KERNEL_OF[dom]} ({dom})",
            "launches_per_step": d["launches"],
            "mean_launch_ms": d["mean_launch_ms"],
            "achieved": d["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": d["frac_hbm"],
            "traffic": measured_traffic("batch", dom),
            "copy_ceiling_gbs": round(copy_gbs, 1),
            "frac_of_copy_ceiling": d["frac_copy"],
        },
        "cpu_baseline": cpu,
        "per_variant": per_variant,
        "stats_ms": round(stats_ms, 4),
        "candidates_only": cand,
        "exhaustive_path": opt,
        "fp16_storage": fp16,
        "wall_s_timed": round(wall, 3),
        "gen_s": round(t_gen, 1),
    }


def workload_uneven(args):
    import torch
    from paper_1812_02647_amd import hrms as H
    from paper_1812_02647_amd import synth
    lengths, hmax = synth.uneven_lengths(512)
    x, offsets, combs = synth.batch(512, lengths, seed=synth.SEED_BASE + 3, comb_fraction=0.05)
    xd = torch.from_numpy(x).cuda()
    total = int(offsets[-1])
    handle = H.hrms_create(0)
    res = {}
    for v in range(4):
        b = H.Batch1D(xd, offsets, v, hmax)
        shape = H.hrms_autotune_1d(handle, b.args, reps=2)
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            b.run(handle, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            b.run(handle, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        batched = e0.elapsed_time(e1) / args.steps
        per = per_spectrum_uneven(H, xd, offsets, v, hmax)
        res[VARIANT_NAMES[v]] = {"batched_ms": round(batched, 3), "per_spectrum_ms": round(per, 3),
                                 "speedup": round(per / batched, 2), "tuned_shape": shape}
    H.hrms_destroy(handle)
    tot = sum(r["batched_ms"] for r in res.values())
    return {"metric": METRIC, "value": round(total / (tot * 1e-3) / 1e9, 3),
            "unit": "G input bins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(tot, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "uneven 1D batch: 512 spectra, lengths log-uniform 2^14..2^23, "
                                   "Hmax in {8,16,32}, 5% combs; one graph-captured persistent "
                                   "launch per variant vs per-spectrum launches",
                       "total_bins": total},
            "per_variant": res}


def per_spectrum_uneven(H, xd, offsets, v, hmax):
    import torch
    old = os.environ.get("HRMS_NO_GRAPH")
    os.environ["HRMS_NO_GRAPH"] = "1"
    try:
        h = H.hrms_create(0)
    finally:
        if old is None:
            os.environ.pop("HRMS_NO_GRAPH")
        else:
            os.environ["HRMS_NO_GRAPH"] = old
    # each spectrum in a slot of its own, 16-byte aligned, as separately
    # allocated spectra would be
    lens = np.diff(offsets)
    slot = np.concatenate([[0], np.cumsum((lens + 3) // 4 * 4)])
    xp = torch.empty(int(slot[-1]), dtype=xd.dtype, device=xd.device)
    batches = []
    for s in range(offsets.size - 1):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        xp[slot[s]:slot[s] + hi - lo].copy_(xd[lo:hi])
        batches.append(H.Batch1D(xp[slot[s]:slot[s] + hi - lo], np.array([0, hi - lo]), v,
                                 int(hmax[s])))
    stream = torch.cuda.current_stream()
    for b in batches:
        b.run(h, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for b in batches:
        b.run(h, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    H.hrms_destroy(h)
    return e0.elapsed_time(e1)


def workload_plane(args):
    import torch
    from paper_1812_02647_amd import hrms as H
    from paper_1812_02647_amd import synth
    zmax, nf, hmax = 42, 1 << 21, 16
    x, combs = synth.plane(nf=nf, zmax=zmax)
    xd = torch.from_numpy(x).cuda()
    rows = 2 * zmax + 1
    handle = H.hrms_create(0)
    names = {H.HRMS_EQ1: "eq1", H.HRMS_MAX: "max", H.HRMS_FREQBIN: "freqbin",
             H.HRMS_GREEDY: "greedy", H.HRMS_GREEDY_FDOT: "greedy_fdot"}

    def timed(plane, dtype_code, stats=None):
        res = {}
        for v in names:
            a = H.hrms_run2d_args()
            a.nf, a.zmax, a.hmax, a.variant, a.ld, a.out_mask = nf, zmax, hmax, v, nf, 7
            a.dtype = dtype_code
            offs, tot = H.hrms_layout_2d(a)
            st = stats if stats is not None else torch.zeros(2, dtype=torch.float64,
                                                             device="cuda")
            a.stats_mode = H.HRMS_STATS_PROVIDED if stats is not None else H.HRMS_STATS_COMPUTE
            hb = torch.empty(tot, dtype=torch.float32, device="cuda")
            ms = torch.empty(rows * nf, dtype=torch.float32, device="cuda")
            bh = torch.empty(rows * nf, dtype=torch.uint8, device="cuda")
            a.x, a.stats, a.h, a.max_snr, a.best_h = (plane.data_ptr(), st.data_ptr(),
                                                      hb.data_ptr(), ms.data_ptr(), bh.data_ptr())
            stream = torch.cuda.current_stream()
            for _ in range(args.warmup):
                H.hrms_run_2d(handle, a, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                H.hrms_run_2d(handle, a, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / args.steps
            byts = rows * nf * plane.element_size() + 4 * tot + 5 * rows * nf
            res[names[v]] = {"ms": round(t, 4), "gbins_per_s": round(rows * nf / t / 1e6, 2),
                             "alg_bytes": byts, "frac_hbm": round(byts / t / 1e9 / 8.0, 4),
                             "traffic": measured_traffic(
                                 "plane", names[v], "f32" if plane.element_size() == 4 else "f16")}
            del hb, ms, bh
        return res

    res = timed(xd, H.HRMS_F32)
    tot_ms = sum(r["ms"] for r in res.values())
    # precision form: the plane normalised to unit mean and stored as FP16
    # (one spectrum of rows x nf bins), statistics (1, sigma / mu) provided
    off = np.array([0, rows * nf], np.int64)
    y = torch.empty(rows * nf, dtype=torch.float16, device="cuda")
    st_raw = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    st_out = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    qa = H.hrms_quantize_args()
    qa.n_spectra, qa.dtype, qa.stats_mode = 1, H.HRMS_F16, H.HRMS_STATS_COMPUTE
    qa.x, qa.offsets, qa.stats, qa.stats_out, qa.y = (xd.data_ptr(), off.ctypes.data,
                                                       st_raw.data_ptr(), st_out.data_ptr(),
                                                       y.data_ptr())
    H.hrms_quantize(handle, qa)
    torch.cuda.synchronize()
    res16 = timed(y, H.HRMS_F16, stats=st_out.reshape(2))
    tot16 = sum(r["ms"] for r in res16.values())
    if args.calibrate_copy and args.workload == "plane":
        c = torch.empty_like(xd)
        c.copy_(xd)
        torch.cuda.synchronize()
        del c
    H.hrms_destroy(handle)
    return {"metric": METRIC, "value": round(rows * nf / tot_ms / 1e6, 3),
            "unit": "G input bins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(tot_ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "2D f-fdot plane 85 x 2^21 FP32, 20 accelerated combs, "
                                   "Hmax=16, eq. (1), Max, freq-bin, Greedy, Greedy with fdot "
                                   "drift (statistics included)"},
            "per_variant": res,
            "fp16_storage": {"value": round(rows * nf / tot16 / 1e6, 3), "unit": "G input bins/s",
                             "ms_per_step": round(tot16, 4), "per_variant": res16,
                             "speedup_vs_fp32": round(tot_ms / tot16, 3)}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the harmonic sum of "
              "independent spectra shards by spectrum with no exchange, which this "
              "single-GPU build does not launch.", file=sys.stderr)
        sys.exit(2)
    fn = {"batch": workload_batch, "uneven": workload_uneven, "plane": workload_plane}
    out = fn[args.workload](args)
    if args.workload == "batch" and not args.no_sub:
        # the other two workloads, reported beside the 1D batch's line
        import torch
        torch.cuda.empty_cache()
        for name in ("plane", "uneven"):
            sub = fn[name](args)
            out[name] = {k: sub[k] for k in ("value", "unit", "ms_per_step", "config",
                                             "per_variant") if k in sub}
            for k in ("fp16_storage",):
                if k in sub:
                    out[name][k] = sub[k]
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
