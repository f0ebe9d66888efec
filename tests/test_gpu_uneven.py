"""The uneven batch at its full size, run as the benchmark runs it: 512 spectra
with lengths log-uniform in 2^14..2^23 and Hmax drawn from {8, 16, 32} per
spectrum, 5% carrying a comb, in one graph-captured launch sequence with the
launch shape chosen by the autotuner.

Sampled outputs of the longest, the shortest and random spectra are compared
with the CPU oracle bit for bit (sums, SNR, best level; statistics and
constants as in the other parity tests), on a graph replay whose outputs were
cleared after the capture run; a few spectra run alone equal their batched
outputs bit for bit.
"""
import numpy as np
import pytest

from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, case_log, check_spectrum, fetch, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    lengths, hmax = synth.uneven_lengths(512)
    x, offsets, combs = synth.batch(512, lengths, seed=synth.SEED_BASE + 3, comb_fraction=0.05)
    xd = torch.from_numpy(x).to("cuda")
    seen = x.astype(np.float64)
    yield xd, seen, offsets, hmax, combs
    del xd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_uneven_batch_full_size(batch, variant):
    import torch
    from paper_1812_02647_amd import hrms as H
    xd, seen, offsets, hmax, _ = batch
    ns = offsets.size - 1
    lens = np.diff(offsets)
    h = H.hrms_create(0)
    try:
        case_log(f"uneven batch variant={NAMES[variant]} 512 spectra 2^14..2^23, autotune")
        b = H.Batch1D(xd, offsets, variant, hmax)
        shape = H.hrms_autotune_1d(h, b.args, reps=1)
        case_log(f"uneven batch variant={NAMES[variant]} tuned shape {shape}, capture + replay")
        b.run(h)
        torch.cuda.synchronize()
        b.h.fill_(float("nan"))
        b.max_snr.fill_(float("nan"))
        b.best_h.fill_(255)
        b.consts.fill_(float("nan"))
        b.stats.fill_(float("nan"))
        b.run(h)                      # the replay must write everything again
        torch.cuda.synchronize()
        out = fetch(b)
        order = np.argsort(lens)
        rng = np.random.default_rng(variant)
        picks = sorted(set(order[-6:].tolist() + order[:6].tolist()
                           + rng.choice(ns, 8, replace=False).tolist()))
        for s in picks:
            idx = sample_indices(int(lens[s]), int(hmax[s]), 1500, rng)
            check_spectrum(b, out, seen, s, variant, int(hmax[s]), idx=idx, check_f64=False,
                           label=f"uneven-{NAMES[variant]}")
        # spectra alone, 16-byte aligned copies: the same bits as in the batch
        for s in (int(order[-1]), int(order[0]), int(picks[len(picks) // 2])):
            lo, hi = int(offsets[s]), int(offsets[s + 1])
            xs = torch.empty(hi - lo, dtype=xd.dtype, device=xd.device)
            xs.copy_(xd[lo:hi])
            one = H.Batch1D(xs, np.array([0, hi - lo], np.int64), variant, int(hmax[s])).run(h)
            torch.cuda.synchronize()
            nl = int(np.log2(int(hmax[s]))) + 1
            for l in range(nl):
                a = b.level(s, l).cpu().numpy()
                c = one.level(0, l).cpu().numpy()
                assert np.array_equal(a.view(np.uint32), c.view(np.uint32)), (s, l)
            assert np.array_equal(out["max_snr"][lo:hi].view(np.uint32),
                                  one.max_snr.cpu().numpy().view(np.uint32)), s
            assert np.array_equal(out["best_h"][lo:hi], one.best_h.cpu().numpy()), s
    finally:
        H.hrms_destroy(h)
