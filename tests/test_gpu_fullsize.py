"""GPU parity at the full size of the 1D batch: 1000 spectra of 2^21 bins,
Hmax = 32, run the way a benchmark step runs it (one statistics pass over the
whole batch, then each of eq. (1)-(4) with those statistics provided and every
output requested, in the default launch shapes of one persistent launch).

The oracle cannot evaluate 2^31 bins, so a few spectra (both ends of the
batch, every spectrum carrying a comb, two at random) are checked on sampled
outputs: both ends, every level boundary, the low bins that hold all 32
harmonics, the bins around each comb's harmonics, and a uniform sample. Only
the sampled outputs are copied back from the device.

Bar: statistics within 1e-12 relative of the oracle's; SNR constants, sums,
maximum SNR and best level bit-identical to the oracle's FP32 evaluation;
sums within 1e-5 relative of the binary64 oracle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, REL_TOL_F64, case_log, sample_indices

pytestmark = pytest.mark.gpu

NS, NB, HMAX = 1000, 1 << 21, 32


@pytest.fixture(scope="module")
def handle():
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    yield h
    H.hrms_destroy(h)


@pytest.fixture(scope="module")
def host_batch():
    x, offsets, combs = synth.batch(NS, NB, seed=synth.SEED_BASE + 1)
    return x, offsets, combs


@pytest.fixture(scope="module", params=["f32", "f16"])
def device_batch(request, host_batch, handle):
    """(dtype, device input, host copy of the stored values as a torch tensor,
    device statistics of the batch). FP16 storage is the plain conversion of
    the same values, made on the host."""
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets, _ = host_batch
    t = torch.from_numpy(x)
    if request.param == "f16":
        t = t.to(torch.float16)
    case_log(f"fullsize stats pass dtype={request.param} {NS}x{NB}")
    xd = t.to("cuda")
    st = H.Batch1D(xd, offsets, 0, HMAX, out_mask=0, want_consts=False).run(handle)
    torch.cuda.synchronize()
    yield request.param, xd, t, st.stats
    del xd, st
    torch.cuda.empty_cache()


def checked_spectra(combs):
    rng = np.random.default_rng(5)
    pick = {0, NS - 1} | {s for s, _ in combs}
    pick |= set(rng.integers(1, NS - 1, size=2).tolist())
    return sorted(pick)


def sampled(s, combs):
    idx = set(sample_indices(NB, HMAX, 1500, np.random.default_rng(1000 + s)).tolist())
    for cs, f0 in combs:
        if cs != s:
            continue
        for k in range(1, 2 * HMAX + 1):
            c = int(math.floor(k * f0))
            for b in (c // HMAX, c // 8, c // 2, c):
                idx.update(j for j in range(b - 2, b + 3) if 0 <= j < NB)
    return np.array(sorted(idx), dtype=np.int64)


def gather(t, pos):
    import torch
    return t[torch.from_numpy(pos).to(t.device)].cpu().numpy()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_fullsize_batch_sampled(handle, host_batch, device_batch, variant):
    import torch
    from paper_1812_02647_amd import hrms as H
    _, offsets, combs = host_batch
    dtype, xd, t, stats = device_batch
    case_log(f"fullsize variant={NAMES[variant]} dtype={dtype} {NS}x{NB} Hmax={HMAX}")
    b = H.Batch1D(xd, offsets, variant, HMAX, out_mask=H.HRMS_OUT_ALL, stats=stats).run(handle)
    torch.cuda.synchronize()
    g_stats = stats.cpu().numpy()
    g_consts = b.consts.cpu().numpy()
    nl = O.num_levels(HMAX)
    for s in checked_spectra(combs):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        xs = t[lo:hi].to(torch.float64).numpy()
        mu, sd = O.stats(xs)
        assert abs(g_stats[s, 0] - mu) <= 1e-12 * abs(mu), (s, g_stats[s], mu)
        assert abs(g_stats[s, 1] - sd) <= 1e-12 * abs(sd), (s, g_stats[s], sd)
        m32, q32, _, _ = O.snr_consts(variant, mu, sd, HMAX)
        assert np.array_equal(g_consts[s, :nl, 0], m32), s
        assert np.array_equal(g_consts[s, :nl, 1], q32), s
        idx = sampled(s, combs)
        h32, ms32, bh32, _ = O.hrms_1d(xs, variant, HMAX, idx=idx, f32=True, mu=mu, sigma=sd)
        h64, _, _, _ = O.hrms_1d(xs, variant, HMAX, idx=idx, f32=False, want_snr=False)
        for l in range(nl):
            ln = NB if variant == O.EQ1 else NB >> l
            valid = idx < ln
            got = gather(b.h, int(b.plane_offsets[s, l]) + idx[valid]).astype(np.float64)
            bad = np.nonzero(got != h32[l][valid])[0]
            assert bad.size == 0, (s, l, idx[valid][bad[:5]], got[bad[:5]], h32[l][valid][bad[:5]])
            ref = h64[l][valid]
            rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)
            assert rel.max() <= REL_TOL_F64, (s, l, rel.max())
        got = gather(b.max_snr, lo + idx).astype(np.float64)
        bad = np.nonzero(got != ms32)[0]
        assert bad.size == 0, (s, idx[bad[:5]], got[bad[:5]], ms32[bad[:5]])
        got = gather(b.best_h, lo + idx)
        bad = np.nonzero(got != bh32)[0]
        assert bad.size == 0, (s, idx[bad[:5]], got[bad[:5]], bh32[bad[:5]])
    del b
