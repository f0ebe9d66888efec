"""hrms_run_1d_noalloc, the 1D entry point that allocates nothing, against
hrms_run_1d through the C ABI: every output bit for bit, on two calls in a row
(the second with a smaller batch, so that the static scratch holds the first
call's tables when it starts), plus the rejection of a batch whose plan does
not fit the scratch. Collected last, so that a failure here hides no other
test."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, case_log, check_spectrum, fetch, to_device_input

pytestmark = pytest.mark.gpu

# (lengths, per-spectrum Hmax): the second batch is smaller in every sense
BATCHES = [
    ([1 << 17, 70001, 1 << 16, 40000, 333, 1], [32, 16, 32, 8, 4, 32]),
    ([50021, 4099], [16, 32]),
]


def _outputs(variant):
    from paper_1812_02647_amd import hrms as H
    if variant == H.HRMS_OPT:
        return H.HRMS_OUT_H
    return H.HRMS_OUT_ALL


def _same(a, b):
    if a is None or b is None:
        return a is None and b is None
    return np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_noalloc_equals_run_1d_twice(variant):
    import torch
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    try:
        for k, (lengths, hmax) in enumerate(BATCHES):
            x, offsets, _ = synth.batch(len(lengths), lengths, seed=700 + k, comb_fraction=0.5)
            xd, seen = to_device_input(x, "f32")
            hm = np.array(hmax, np.uint8)
            om = _outputs(variant)
            case_log(f"noalloc call {k} variant={NAMES[variant]} lengths={lengths}")
            ref = H.Batch1D(xd, offsets, variant, hm, out_mask=om).run(h)
            got = H.Batch1D(xd, offsets, variant, hm, out_mask=om).run_noalloc(h)
            torch.cuda.synchronize()
            r, g = fetch(ref), fetch(got)
            for key in ("stats", "consts", "h", "max_snr", "best_h"):
                assert _same(r[key], g[key]), (k, key)
            # and one spectrum against the oracle, so that the comparison is
            # not between two equally wrong results
            if variant != H.HRMS_OPT:
                check_spectrum(got, g, seen, len(lengths) - 1, variant, hmax[-1],
                               check_f64=False, label=f"noalloc{k}")
            else:
                n = lengths[-1]
                ref_h, _, _, _ = O.hrms_1d(seen[int(offsets[-2]):], O.OPT, hmax[-1], f32=True,
                                           want_snr=False)
                for l in range(O.num_levels(hmax[-1])):
                    lv = got.level(len(lengths) - 1, l).cpu().numpy().astype(np.float64)
                    assert np.array_equal(lv, ref_h[l][:n >> l]), (k, l)
    finally:
        H.hrms_destroy(h)


def test_noalloc_candidates_twice():
    """The candidate list (its counter is cleared by the constants kernel,
    not by a memset) is the same set from both entry points, twice."""
    import torch
    from paper_1812_02647_amd import hrms as H
    h = H.hrms_create(0)
    try:
        for k, (lengths, hmax) in enumerate(BATCHES):
            x, offsets, _ = synth.batch(len(lengths), lengths, seed=710 + k, comb_fraction=1.0)
            xd, _ = to_device_input(x, "f32")
            case_log(f"noalloc candidates call {k} lengths={lengths}")
            om = H.HRMS_OUT_CAND
            ref = H.Batch1D(xd, offsets, H.HRMS_GREEDY, 32, out_mask=om, cand_capacity=1 << 16,
                            cand_threshold=4.0).run(h)
            got = H.Batch1D(xd, offsets, H.HRMS_GREEDY, 32, out_mask=om, cand_capacity=1 << 16,
                            cand_threshold=4.0).run_noalloc(h)
            torch.cuda.synchronize()
            nr, rr = ref.candidates()
            ng, rg = got.candidates()
            assert nr == ng and nr > 0, (k, nr, ng)
            assert nr <= 1 << 16
            assert np.array_equal(np.sort(rr, order=["spectrum", "bin"]),
                                  np.sort(rg, order=["spectrum", "bin"])), k
    finally:
        H.hrms_destroy(h)


def test_noalloc_rejects_a_plan_larger_than_its_scratch():
    """300 000 one-bin spectra need about 70 MB of tables and constants, more
    than the 48 MiB scratch: rejected before anything is enqueued (the outputs
    keep their fill), while hrms_run_1d runs the same batch."""
    import torch
    from paper_1812_02647_amd import hrms as H
    n = 300_000
    offsets = np.arange(n + 1, dtype=np.int64)
    xd = torch.rand(n, dtype=torch.float32, device="cuda") + 0.5
    h = H.hrms_create(0)
    try:
        case_log(f"noalloc oversize n_spectra={n}")
        b = H.Batch1D(xd, offsets, H.HRMS_FREQBIN, 1, want_consts=False)
        b.max_snr.fill_(-7.0)
        torch.cuda.synchronize()
        with pytest.raises(H.HrmsError) as ei:
            b.run_noalloc(h)
        assert ei.value.status == H.HRMS_E_INVAL
        assert "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((b.max_snr == -7.0).all())
        b.run(h)
        torch.cuda.synchronize()
        # one-bin spectra: sigma 0, so every SNR is 0
        assert bool((b.max_snr == 0.0).all())
        assert bool((b.h == xd).all())
    finally:
        H.hrms_destroy(h)
