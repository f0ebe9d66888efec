"""GPU parity of the 1D harmonic sum (eq. (1)-(4), arXiv:1812.02647) against
the CPU oracle, through the C ABI.

Bar: sums, SNR and best level bit-identical to the oracle's FP32 evaluation;
sums within 1e-5 relative of the binary64 oracle; statistics within 1e-12.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import (NAMES, case_log, check_spectrum, fetch, run_1d, sample_indices,
                               to_device_input)

pytestmark = pytest.mark.gpu
VARIANTS = [0, 1, 2, 3]


@pytest.fixture(scope="module")
def handle():
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    yield h
    H.hrms_destroy(h)


@pytest.mark.parametrize("variant", VARIANTS)
def test_single_spectrum_comb(handle, variant):
    """N = 65536 exponential noise + on-bin comb at bin 1000 (8 harmonics,
    amplitude 20/i), Hmax = 8: every output compared."""
    x = synth.single_spectrum()
    offsets = np.array([0, x.size], np.int64)
    xd, seen = to_device_input(x, "f32")
    case_log(f"single_spectrum_comb variant={NAMES[variant]} N={x.size} hmax=8")
    b = run_1d(handle, xd, offsets, variant, 8)
    out = fetch(b)
    check_spectrum(b, out, seen, 0, variant, 8, label="c1")
    ms = out["max_snr"]
    if variant == O.FREQBIN:
        assert int(np.argmax(ms)) == 1000
    if variant == O.EQ1:
        top = int(np.argmax(ms))
        assert top // int(out["best_h"][top]) == 1000


RAGGED_LEN = [1, 2, 3, 5, 31, 33, 64, 4097, 70001, 200003]
RAGGED_HMAX = [1, 2, 4, 32, 8, 16, 32, 32, 32, 32]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_ragged_batch(handle, variant, dtype):
    """Uneven lengths (down to 1 bin), misaligned packing, per-spectrum Hmax;
    many tiles and ragged tails; every output compared."""
    x, offsets, _ = synth.batch(len(RAGGED_LEN), RAGGED_LEN, seed=77, comb_fraction=0.0)
    xd, seen = to_device_input(x, dtype)
    case_log(f"ragged_batch variant={NAMES[variant]} dtype={dtype} lengths={RAGGED_LEN}")
    b = run_1d(handle, xd, offsets, variant, np.array(RAGGED_HMAX, np.uint8))
    out = fetch(b)
    for s, hm in enumerate(RAGGED_HMAX):
        check_spectrum(b, out, seen, s, variant, hm, label=f"ragged-{dtype}",
                       check_f64=(dtype == "f32"))


@pytest.mark.parametrize("variant", VARIANTS)
def test_integer_valued_inputs_match_binary64(handle, variant):
    """Integer bins: every partial sum is exact in FP32, so the device equals
    the binary64 oracle bit for bit on S (independently of summation order)."""
    rng = np.random.default_rng(5)
    lengths = [5000, 131072, 777]
    x = rng.integers(0, 200, size=sum(lengths)).astype(np.float32)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    xd, seen = to_device_input(x, "f32")
    case_log(f"integer_inputs variant={NAMES[variant]}")
    b = run_1d(handle, xd, offsets, variant, 32, out_mask=1)
    h = b.h.cpu().numpy()
    for s in range(len(lengths)):
        xs = seen[offsets[s]:offsets[s + 1]]
        h64, _, _, _ = O.hrms_1d(xs, variant, 32, f32=False, want_snr=False)
        for l in range(6):
            ln = lengths[s] if variant == 0 else lengths[s] >> l
            plane = h[b.plane_offsets[s, l]:b.plane_offsets[s, l] + ln].astype(np.float64)
            S_dev = np.round(plane / np.float32(1.0 / math.sqrt(1 << l)))
            S_ref = np.round(h64[l][:ln] * math.sqrt(1 << l))
            assert np.array_equal(S_dev, S_ref), (s, l)


@pytest.mark.parametrize("variant", VARIANTS)
def test_stats_provided(handle, variant):
    import torch
    x, offsets, _ = synth.batch(3, [10000, 20011, 4096], seed=9, comb_fraction=0.0)
    xd, seen = to_device_input(x, "f32")
    st = np.array([[1.25, 0.75], [0.5, 2.0], [1.0, 0.0]])
    stats = torch.from_numpy(st).to("cuda")
    case_log(f"stats_provided variant={NAMES[variant]}")
    b = run_1d(handle, xd, offsets, variant, 16, stats=stats)
    out = fetch(b)
    assert np.array_equal(out["stats"], st)  # read, not written
    for s in range(3):
        check_spectrum(b, out, seen, s, variant, 16, stats_provided=tuple(st[s]),
                       label="provided")
    # sigma = 0 -> q = 0: every SNR is 0 and ties keep H = 1
    lo, hi = offsets[2], offsets[3]
    assert np.all(out["max_snr"][lo:hi] == 0) and np.all(out["best_h"][lo:hi] == 1)


@pytest.mark.parametrize("mask", [1, 2, 4, 6])
def test_output_subsets(handle, mask):
    x, offsets, _ = synth.batch(2, [30000, 12345], seed=11, comb_fraction=0.0)
    xd, seen = to_device_input(x, "f32")
    case_log(f"output_subsets mask={mask}")
    full = fetch(run_1d(handle, xd, offsets, 1, 32))
    b = run_1d(handle, xd, offsets, 1, 32, out_mask=mask)
    part = fetch(b)
    for k in ("h", "max_snr", "best_h"):
        if part[k] is not None:
            assert np.array_equal(part[k], full[k][:part[k].size])


@pytest.mark.parametrize("variant", VARIANTS)
def test_repeatable_bitwise(handle, variant):
    """Two runs of the same batch give identical bits (statistics included)."""
    x, offsets, _ = synth.batch(5, [300000, 1 << 18, 99991, 5, 70000], seed=13)
    xd, _ = to_device_input(x, "f32")
    case_log(f"repeatable variant={NAMES[variant]}")
    a = fetch(run_1d(handle, xd, offsets, variant, 32))
    b = fetch(run_1d(handle, xd, offsets, variant, 32))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("variant", VARIANTS)
def test_batched_equals_per_spectrum(handle, variant):
    """One persistent launch over an uneven batch gives the same bits as one
    launch per spectrum."""
    lengths, hmax = synth.uneven_lengths(24, seed=3, lo_exp=10, hi_exp=17)
    x, offsets, _ = synth.batch(len(lengths), lengths, seed=21, comb_fraction=0.1)
    xd, _ = to_device_input(x, "f32")
    case_log(f"batched_vs_per_spectrum variant={NAMES[variant]} n=24")
    whole = fetch(run_1d(handle, xd, offsets, variant, hmax))
    bw = run_1d(handle, xd, offsets, variant, hmax)
    for s in range(len(lengths)):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        one = run_1d(handle, xd[lo:hi].clone(), np.array([0, hi - lo]), variant, int(hmax[s]))
        o = fetch(one)
        assert np.array_equal(o["max_snr"], whole["max_snr"][lo:hi])
        assert np.array_equal(o["best_h"], whole["best_h"][lo:hi])
        assert np.array_equal(o["stats"][0], whole["stats"][s])
        for l in range(O.num_levels(int(hmax[s]))):
            ln = (hi - lo) if variant == 0 else (hi - lo) >> l
            pw = whole["h"][bw.plane_offsets[s, l]:bw.plane_offsets[s, l] + ln]
            po = o["h"][one.plane_offsets[0, l]:one.plane_offsets[0, l] + ln]
            assert np.array_equal(pw, po), (s, l)


@pytest.mark.parametrize("variant", VARIANTS)
def test_long_spectrum_sampled(handle, variant):
    """One 2^23-bin spectrum (the largest of the uneven batch), Hmax = 32,
    sampled outputs."""
    N = 1 << 23
    x, offsets, _ = synth.batch(1, [N], seed=31, comb_fraction=1.0)
    xd, seen = to_device_input(x, "f32")
    case_log(f"long_spectrum variant={NAMES[variant]} N={N}")
    b = run_1d(handle, xd, offsets, variant, 32)
    out = fetch(b)
    idx = sample_indices(N, 32, 4000, np.random.default_rng(variant))
    check_spectrum(b, out, seen, 0, variant, 32, idx=idx, label="long")


def _same_or_both_nan(got, exp):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    return (got == exp) | (np.isnan(got) & np.isnan(exp))


@pytest.mark.parametrize("variant", VARIANTS)
def test_nan_and_inf_bins(handle, variant):
    """Non-finite bins are outside the method's domain; the run must still
    finish and give exactly what the definitions give in IEEE arithmetic:
    comparisons with NaN are false, so a Max window keeps its first bin's NaN
    and skips later ones, Greedy stays on the left bin of a NaN pair, and a
    sum that meets NaN or +inf carries it. Statistics are provided (those of
    the clean spectrum), so the constants stay finite."""
    from paper_1812_02647_amd import hrms as H
    import torch
    n = 20011
    x = synth.exponential(99, 0, n).astype(np.float32)
    mu, sd = O.stats(x.astype(np.float64))
    for pos in (0, 1, 7, 64, 65, 129, 500, 1001, 4000, 9999, n - 1):
        x[pos] = np.nan
    for pos in (3, 66, 250, 2048, 7777, n - 2):
        x[pos] = np.inf
    offsets = np.array([0, n], np.int64)
    xd, seen = to_device_input(x, "f32")
    case_log(f"nan_and_inf_bins variant={NAMES[variant]} N={n} hmax=32")
    st = torch.tensor([[mu, sd]], dtype=torch.float64, device="cuda")
    b = run_1d(handle, xd, offsets, variant, 32, stats=st)
    out = fetch(b)
    h32, ms32, bh32, _ = O.hrms_1d(seen, variant, 32, f32=True, mu=mu, sigma=sd)
    for l in range(6):
        ln = n if variant == 0 else n >> l
        got = out["h"][int(b.plane_offsets[0, l]):int(b.plane_offsets[0, l]) + ln]
        ok = _same_or_both_nan(got, h32[l][:ln])
        assert ok.all(), (l, np.nonzero(~ok)[0][:5])
    assert _same_or_both_nan(out["max_snr"], ms32).all()
    assert np.array_equal(out["best_h"], bh32)


@pytest.mark.parametrize("variant", VARIANTS)
def test_two_streams_same_signature(variant):
    """Two batches with the same offsets (so the same cached plan and its
    scratch) but different bins, run alternately on two streams of one handle
    without synchronising in between: each result equals the oracle."""
    import torch
    from paper_1812_02647_amd import hrms as H
    lengths = [1 << 17, 70001, 1 << 16, 40000]
    xa, offsets, _ = synth.batch(len(lengths), lengths, seed=401, comb_fraction=0.0)
    xb, offsets_b, _ = synth.batch(len(lengths), lengths, seed=402, comb_fraction=0.0)
    assert np.array_equal(offsets, offsets_b)
    da, seen_a = to_device_input(xa, "f32")
    db, seen_b = to_device_input(xb, "f32")
    h = H.hrms_create(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        case_log(f"two_streams_same_signature variant={NAMES[variant]} lengths={lengths}")
        ba = H.Batch1D(da, offsets, variant, 32)
        bb = H.Batch1D(db, offsets, variant, 32)
        torch.cuda.synchronize()
        for _ in range(3):
            ba.run(h, s1)
            bb.run(h, s2)
        torch.cuda.synchronize()
        for b, seen in ((ba, seen_a), (bb, seen_b)):
            out = fetch(b)
            for s in range(len(lengths)):
                idx = sample_indices(lengths[s], 32, 2000, np.random.default_rng(s))
                check_spectrum(b, out, seen, s, variant, 32, idx=idx, check_f64=False,
                               label="two-streams")
    finally:
        H.hrms_destroy(h)
