"""Precision form (FP16 / BF16 storage, FP32 accumulation), GPU vs oracle.

1. hrms_quantize: y = round(x * fl32(1/mu)) to FP16 (round to nearest even,
   saturating at 65504) or BF16 (round to nearest even) equals the oracle's
   binary32 product rounded by numpy (FP16) or by torch's CPU conversion
   (BF16), bit for bit, and (mu', sigma') = (1, sigma / mu).
2. Error of the narrow-storage sums against the binary64 oracle on the
   unquantised normalised spectrum: for non-negative inputs eq. (1), eq. (3)
   and eq. (2) stay within (u/2 + (H + 2) 2^-24) |h| + H 2^-25 (u = 2^-10
   for FP16, 2^-7 for BF16: each stored bin is within u/2 of its value in the
   normal range and within 2^-25 absolute below it, FP16's subnormals; the
   FP32 scaling, accumulation and 1/sqrt(H) factor add 2^-24 each per term;
   sums of non-negative terms and maxima keep the bound); Greedy may follow
   another path, so its error is only reported.
3. Candidate lists {n : max_snr >= 6} of narrow storage and FP32 storage
   mostly agree, and every injected comb that FP32 storage finds is found.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, case_log, fetch, run_1d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    yield h
    H.hrms_destroy(h)


def quantize(handle, xdev, offsets, dtype, stats=None):
    import torch
    from paper_1812_02647_amd import hrms as H
    n = offsets.size - 1
    a = H.hrms_quantize_args()
    a.n_spectra = n
    a.dtype = H.HRMS_F16 if dtype == "f16" else H.HRMS_BF16
    a.stats_mode = 1 if stats is not None else 0
    a.x = xdev.data_ptr()
    off = np.ascontiguousarray(offsets, np.int64)
    a.offsets = off.ctypes.data
    st = stats if stats is not None else torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    so = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    y = torch.empty(int(offsets[-1]), dtype=torch.float16 if dtype == "f16" else torch.bfloat16,
                    device="cuda")
    a.stats, a.stats_out, a.y = st.data_ptr(), so.data_ptr(), y.data_ptr()
    H.hrms_quantize(handle, a)
    torch.cuda.synchronize()
    return y, st.cpu().numpy(), so.cpu().numpy()


def reference_narrow(y32, dtype):
    import torch
    if dtype == "f16":
        return np.clip(y32, -65504.0, 65504.0).astype(np.float32).astype(np.float16)
    return torch.from_numpy(y32.astype(np.float32)).to(torch.bfloat16)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_quantize_bits(handle, dtype):
    import torch
    x, offsets, _ = synth.batch(5, [1000, 65536, 3, 77777, 5000], seed=61, comb_fraction=0.4)
    x = x.copy()
    x[10] = 3.0e9          # saturates in FP16 once scaled
    x[11] = 0.0
    x[12] = 1e-30          # underflows
    xd = torch.from_numpy(x).to("cuda")
    case_log(f"quantize dtype={dtype}")
    y, st, so = quantize(handle, xd, offsets, dtype)
    for s in range(offsets.size - 1):
        lo, hi = offsets[s], offsets[s + 1]
        xs = x[lo:hi].astype(np.float64)
        mu, sd = O.stats(xs)
        assert abs(st[s, 0] - mu) <= 1e-12 * mu and abs(st[s, 1] - sd) <= 1e-12 * sd
        assert so[s, 0] == 1.0 and abs(so[s, 1] - sd / mu) <= 1e-12 * (sd / mu)
        ref = reference_narrow(O.scale_f32(xs, st[s, 0]), dtype)
        got = y[lo:hi].cpu()
        if dtype == "f16":
            assert np.array_equal(got.numpy().view(np.uint16), ref.view(np.uint16)), s
        else:
            assert torch.equal(got.view(torch.int16), ref.view(torch.int16)), s


def error_study(handle, dtype, variants, u, n_spec=6, nb=1 << 20, hmax=32):
    """Narrow-storage GPU sums vs the binary64 oracle on the exact normalised
    spectrum; returns, per variant and level, the max relative error and the
    max ratio of the error to the bound of item 2."""
    import torch
    x, offsets, _ = synth.batch(n_spec, nb, seed=71, comb_fraction=0.5)
    xd = torch.from_numpy(x).to("cuda")
    y, st, so = quantize(handle, xd, offsets, dtype)
    out = {}
    rng = np.random.default_rng(1)
    for v in variants:
        b = run_1d(handle, y, offsets, v, hmax)
        o = fetch(b)
        worst = np.zeros(O.num_levels(hmax))
        ratio = np.zeros(O.num_levels(hmax))
        for s in range(n_spec):
            lo, hi = offsets[s], offsets[s + 1]
            xs = x[lo:hi].astype(np.float64) / st[s, 0]     # exact normalised spectrum
            # include the smallest bins: FP16 stores those below 2^-14 as subnormals
            idx = np.unique(np.concatenate([np.arange(0, 64), rng.integers(0, nb // hmax, 800),
                                            rng.integers(0, nb, 800),
                                            np.argsort(xs)[:32]])).astype(np.int64)
            h64, _, _, _ = O.hrms_1d(xs, v, hmax, idx=idx, f32=False, want_snr=False)
            for l in range(O.num_levels(hmax)):
                ln = nb if v == 0 else nb >> l
                valid = idx < ln
                got = o["h"][b.plane_offsets[s, l] + idx[valid]].astype(np.float64)
                ref = h64[l][valid]
                err = np.abs(got - ref)
                H = 1 << l
                bound = (u / 2 + (H + 2) * 2.0 ** -24) * np.abs(ref) + H * 2.0 ** -25
                worst[l] = max(worst[l], float(np.max(err / np.maximum(np.abs(ref), 1e-300))))
                ratio[l] = max(ratio[l], float(np.max(err / bound)))
        out[NAMES[v]] = (worst, ratio)
    return out


@pytest.mark.parametrize("dtype,u", [("f16", 2.0 ** -10), ("bf16", 2.0 ** -7)])
def test_narrow_storage_error_bound(handle, dtype, u):
    case_log(f"precision error study dtype={dtype}")
    errs = error_study(handle, dtype, [0, 1, 2, 3], u)
    for name in ("eq1", "max", "freqbin"):
        for l, r in enumerate(errs[name][1]):
            assert r <= 1.0, (dtype, name, 1 << l, r, errs[name][0][l])
    print(f"max relative error vs binary64, {dtype}:",
          {k: [float(f"{e:.3g}") for e in v[0]] for k, v in errs.items()})


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_candidate_lists_agree(handle, dtype):
    """Candidates above SNR 6 from narrow storage vs FP32 storage of the same
    normalised spectra: large overlap (Jaccard) and no loss of the injected
    combs."""
    import torch
    x, offsets, combs = synth.batch(8, 1 << 20, seed=81, comb_fraction=0.5)
    xd = torch.from_numpy(x).to("cuda")
    case_log(f"candidate lists dtype={dtype}")
    y, st, so = quantize(handle, xd, offsets, dtype)
    for v in [0, 1, 2, 3]:
        o16 = fetch(run_1d(handle, y, offsets, v, 32))
        o32 = fetch(run_1d(handle, xd, offsets, v, 32))
        c16 = set(np.nonzero(o16["max_snr"] >= 6.0)[0].tolist())
        c32 = set(np.nonzero(o32["max_snr"] >= 6.0)[0].tolist())
        jac = len(c16 & c32) / max(1, len(c16 | c32))
        assert jac > (0.95 if dtype == "f16" else 0.7), (NAMES[v], dtype, jac)
        # an injected comb found with FP32 storage is found with narrow storage
        for s, f0 in combs:
            if v == 0:
                continue
            near = [offsets[s] + int(math.floor(f0)) + d for d in (-1, 0, 1)]
            if any(n in c32 for n in near):
                assert any(n in c16 for n in near), (NAMES[v], dtype, s, f0)
