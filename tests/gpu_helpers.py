"""Helpers of the GPU parity tests: run the library through its C ABI on torch
device buffers and compare every requested output with the CPU oracle.

Inputs are made on the host (the shared generator), converted to the storage
type on the host, and the oracle receives exactly the values the device reads
(narrow types widened exactly). No expected value comes from the device.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NAMES = {0: "eq1", 1: "max", 2: "freqbin", 3: "greedy", 4: "opt", 5: "greedy_fdot"}
# FP32 relative error bound of the sums against the binary64 oracle
REL_TOL_F64 = 1e-5


def case_log(msg: str) -> None:
    """Names the case about to run on the GPU, before it runs."""
    line = f"[gpu-case] {msg}"
    print(line, file=sys.stderr, flush=True)
    d = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(d):
        with open(os.path.join(d, "gpu_cases.log"), "a") as f:
            f.write(line + "\n")


def to_device_input(x32: np.ndarray, dtype: str):
    """Returns (device tensor, host float64 copy of the values it holds)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x32, np.float32))
    if dtype == "f16":
        t = t.to(torch.float16)
    elif dtype == "bf16":
        t = t.to(torch.bfloat16)
    seen = t.to(torch.float64).numpy()
    return t.to("cuda"), seen


def run_1d(handle, xdev, offsets, variant, hmax, out_mask=7, stats=None):
    import torch
    from paper_1812_02647_amd import hrms as H
    b = H.Batch1D(xdev, offsets, variant, hmax, out_mask=out_mask, stats=stats)
    b.run(handle)
    torch.cuda.synchronize()
    return b


def fetch(b):
    out = {"stats": b.stats.cpu().numpy(), "consts": b.consts.cpu().numpy()}
    out["h"] = b.h.cpu().numpy() if b.h is not None else None
    out["max_snr"] = b.max_snr.cpu().numpy() if b.max_snr is not None else None
    out["best_h"] = b.best_h.cpu().numpy() if b.best_h is not None else None
    return out


def check_spectrum(b, out, seen, s, variant, hmax_s, idx=None, stats_provided=None,
                   check_f64=True, label=""):
    """Compares spectrum s of a finished batch with the oracle.

    Sums, SNR and best level are compared bit for bit with the oracle's FP32
    evaluation (same order, same constants); the sums additionally against the
    binary64 oracle within REL_TOL_F64; statistics within 1e-12 relative."""
    lo, hi = int(b.offsets[s]), int(b.offsets[s + 1])
    xs = seen[lo:hi]
    N = hi - lo
    nl = O.num_levels(hmax_s)
    if stats_provided is None:
        mu, sd = O.stats(xs)
        g_mu, g_sd = out["stats"][s]
        assert abs(g_mu - mu) <= 1e-12 * abs(mu) + 1e-300, (label, s, g_mu, mu)
        assert abs(g_sd - sd) <= 1e-12 * abs(sd) + 1e-300, (label, s, g_sd, sd)
    else:
        mu, sd = stats_provided
    m32, q32, m64, q64 = O.snr_consts(variant, mu, sd, hmax_s)
    gc = out["consts"][s]
    assert np.array_equal(gc[:nl, 0], m32), (label, s, gc[:nl, 0], m32)
    assert np.array_equal(gc[:nl, 1], q32), (label, s, gc[:nl, 1], q32)
    assert np.all(gc[nl:] == 0)
    if idx is None:
        idx = np.arange(N, dtype=np.int64)
    h32, ms32, bh32, _ = O.hrms_1d(xs, variant, hmax_s, idx=idx, f32=True, mu=mu, sigma=sd)
    if out["h"] is not None:
        h64 = None
        if check_f64:
            h64, _, _, _ = O.hrms_1d(xs, variant, hmax_s, idx=idx, f32=False, want_snr=False)
        for l in range(nl):
            plane = out["h"][int(b.plane_offsets[s, l]):]
            ln = N if variant == 0 else N >> l
            valid = idx < ln
            if variant != 0:
                assert np.all(np.isnan(h32[l][~valid]))
            got = plane[idx[valid]].astype(np.float64)
            exp = h32[l][valid]
            bad = np.nonzero(got != exp)[0]
            assert bad.size == 0, (label, "h", s, l, idx[valid][bad[:5]], got[bad[:5]], exp[bad[:5]])
            if h64 is not None and valid.any():
                ref = h64[l][valid]
                rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)
                assert rel.max() <= REL_TOL_F64, (label, "h vs f64", s, l, rel.max())
    if out["max_snr"] is not None:
        got = out["max_snr"][lo + idx].astype(np.float64)
        bad = np.nonzero(got != ms32)[0]
        assert bad.size == 0, (label, "max_snr", s, idx[bad[:5]], got[bad[:5]], ms32[bad[:5]])
    if out["best_h"] is not None:
        got = out["best_h"][lo + idx]
        bad = np.nonzero(got != bh32)[0]
        assert bad.size == 0, (label, "best_h", s, idx[bad[:5]], got[bad[:5]], bh32[bad[:5]])


def sample_indices(N: int, hmax: int, count: int, rng) -> np.ndarray:
    """Outputs the oracle can afford one by one: both ends, every level
    boundary floor(N/H) +- 2, the low bins that carry all harmonics, and a
    uniform sample."""
    pts = set(range(0, min(N, 40)))
    pts.update(range(max(0, N - 40), N))
    H = 1
    while H <= hmax:
        L = N // H
        for d in range(-3, 3):
            if 0 <= L + d < N:
                pts.add(L + d)
        H *= 2
    pts.update(rng.integers(0, max(1, N // max(hmax, 1)), size=count // 2).tolist())
    pts.update(rng.integers(0, N, size=count // 2).tolist())
    return np.array(sorted(pts), dtype=np.int64)
