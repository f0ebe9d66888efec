"""Candidate output (HRMS_OUT_CAND) of the 1D kernels against the oracle.

For each variant, on a ragged batch with injected combs: the set of
(spectrum, bin) records equals the oracle's {n : max_snr >= threshold} per
spectrum, and each record's SNR and best H equal the oracle's bits (FP32
evaluation). The record order is unspecified, so records are compared as a
set. The same run's max_snr output, thresholded, gives the same set; a
capacity smaller than the count keeps the count and writes a subset.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, case_log, fetch

pytestmark = pytest.mark.gpu

THR = 4.5


@pytest.fixture(scope="module")
def handle():
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    yield h
    H.hrms_destroy(h)


def batch():
    lengths = [(1 << 18) + 5, 40000, 3, 131072]
    x, offsets, combs = synth.batch(len(lengths), lengths, seed=53, comb_fraction=0.75)
    return x, offsets


def oracle_set(x, offsets, variant, hmax):
    want = {}
    for s in range(offsets.size - 1):
        xs = x[offsets[s]:offsets[s + 1]].astype(np.float64)
        _, ms, bh, _ = O.hrms_1d(xs, variant, hmax, f32=True)
        bins, snr, hh = O.candidates(ms.astype(np.float32), bh, THR)
        for b, v, hv in zip(bins, snr, hh):
            want[(s, int(b))] = (np.float32(v), int(hv))
    return want


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_candidates_match_oracle(handle, variant):
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets = batch()
    xd = torch.from_numpy(x).to("cuda")
    case_log(f"candidates variant={NAMES[variant]}")
    b = H.Batch1D(xd, offsets, variant, 32, out_mask=H.HRMS_OUT_CAND | H.HRMS_OUT_MAXSNR,
                  cand_capacity=1 << 16, cand_threshold=THR).run(handle)
    torch.cuda.synchronize()
    n, rec = b.candidates()
    assert n == rec.size
    got = {(int(r["spectrum"]), int(r["bin"])): (np.float32(r["snr"]), int(r["best_h"]))
           for r in rec}
    assert len(got) == n                       # no record twice
    want = oracle_set(x, offsets, variant, 32)
    assert set(got) == set(want), (len(got), len(want))
    for k, (snr, hv) in want.items():
        assert got[k][0].view(np.uint32) == snr.view(np.uint32) and got[k][1] == hv, k
    # the same run's max_snr, thresholded, names the same bins
    ms = fetch(b)["max_snr"]
    from_ms = {(s, int(i)) for s in range(offsets.size - 1)
               for i in np.nonzero(ms[offsets[s]:offsets[s + 1]] >= THR)[0]}
    assert from_ms == set(got)


def test_candidate_capacity_overflow(handle):
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets = batch()
    xd = torch.from_numpy(x).to("cuda")
    case_log("candidates overflow")
    full = H.Batch1D(xd, offsets, 2, 32, out_mask=H.HRMS_OUT_CAND, cand_capacity=1 << 16,
                     cand_threshold=THR).run(handle)
    small = H.Batch1D(xd, offsets, 2, 32, out_mask=H.HRMS_OUT_CAND, cand_capacity=5,
                      cand_threshold=THR).run(handle)
    none = H.Batch1D(xd, offsets, 2, 32, out_mask=H.HRMS_OUT_CAND, cand_capacity=0,
                     cand_threshold=THR).run(handle)
    torch.cuda.synchronize()
    n_full, rec_full = full.candidates()
    n_small, rec_small = small.candidates()
    n_none, _ = none.candidates()
    assert n_full > 5 and n_small == n_full and n_none == n_full
    assert rec_small.size == 5
    keys = {(int(r["spectrum"]), int(r["bin"])) for r in rec_full}
    assert all((int(r["spectrum"]), int(r["bin"])) in keys for r in rec_small)


def oracle_peaks(x, offsets, variant, hmax):
    want = {}
    for s in range(offsets.size - 1):
        xs = x[offsets[s]:offsets[s + 1]].astype(np.float64)
        _, ms, bh, _ = O.hrms_1d(xs, variant, hmax, f32=True)
        bins, snr, hh = O.peaks(ms.astype(np.float32), bh, THR)
        for b, v, hv in zip(bins, snr, hh):
            want[(s, int(b))] = (np.float32(v), int(hv))
    return want


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_peaks_match_oracle(handle, variant):
    """HRMS_OUT_PEAKS: the local maxima of max_snr above the threshold, per
    spectrum, as a set equal to the oracle's, SNR and best H bit for bit."""
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets = batch()
    xd = torch.from_numpy(x).to("cuda")
    case_log(f"peaks variant={NAMES[variant]}")
    mask = H.HRMS_OUT_PEAKS | H.HRMS_OUT_MAXSNR | H.HRMS_OUT_BESTH
    b = H.Batch1D(xd, offsets, variant, 32, out_mask=mask, cand_capacity=1 << 16,
                  cand_threshold=THR).run(handle)
    torch.cuda.synchronize()
    n, rec = b.candidates()
    assert n == rec.size
    got = {(int(r["spectrum"]), int(r["bin"])): (np.float32(r["snr"]), int(r["best_h"]))
           for r in rec}
    assert len(got) == n
    want = oracle_peaks(x, offsets, variant, 32)
    assert 0 < len(want) < len(oracle_set(x, offsets, variant, 32))
    assert set(got) == set(want), (len(got), len(want))
    for k, (snr, hv) in want.items():
        assert got[k][0].view(np.uint32) == snr.view(np.uint32) and got[k][1] == hv, k
    # without HRMS_OUT_BESTH the records carry best H = 0
    b2 = H.Batch1D(xd, offsets, variant, 32, out_mask=H.HRMS_OUT_PEAKS | H.HRMS_OUT_MAXSNR,
                   cand_capacity=1 << 16, cand_threshold=THR).run(handle)
    torch.cuda.synchronize()
    n2, rec2 = b2.candidates()
    assert n2 == n and set(int(v) for v in rec2["best_h"]) == {0}
