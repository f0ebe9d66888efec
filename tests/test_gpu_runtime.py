"""Host runtime on the GPU: graph-captured launches, the autotuner and the
tune cache give the same bits as direct launches and the oracle."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth
from tests.gpu_helpers import NAMES, case_log, check_spectrum, fetch, run_1d, to_device_input

pytestmark = pytest.mark.gpu


def make_handle(no_graph=False, tune=None):
    from paper_1812_02647_amd import hrms as H
    old = os.environ.get("HRMS_NO_GRAPH")
    if no_graph:
        os.environ["HRMS_NO_GRAPH"] = "1"
    else:
        os.environ.pop("HRMS_NO_GRAPH", None)
    try:
        return H.hrms_create(0, tune)
    finally:
        if old is None:
            os.environ.pop("HRMS_NO_GRAPH", None)
        else:
            os.environ["HRMS_NO_GRAPH"] = old


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_graph_replays_match_direct_launches(variant):
    """The captured graph is replayed several times, with other work and
    synchronisations in between; every replay equals the direct launch."""
    import torch
    from paper_1812_02647_amd import hrms as H
    lengths, hmax = synth.uneven_lengths(40, seed=5, lo_exp=10, hi_exp=18)
    x, offsets, _ = synth.batch(len(lengths), lengths, seed=17, comb_fraction=0.1)
    xd, seen = to_device_input(x, "f32")
    hg, hd = make_handle(False), make_handle(True)
    try:
        case_log(f"graph replays variant={NAMES[variant]}")
        ref = fetch(run_1d(hd, xd, offsets, variant, hmax))
        b = H.Batch1D(xd, offsets, variant, hmax)
        for rep in range(4):
            for k in ("h", "max_snr", "best_h", "stats", "consts"):
                t = getattr(b, k)
                if t is not None:
                    t.fill_(-7)
            b.run(hg)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
            torch.cuda.synchronize()
            got = fetch(b)
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)
        check_spectrum(b, fetch(b), seen, 0, variant, int(hmax[0]), label="graph")
    finally:
        H.hrms_destroy(hg)
        H.hrms_destroy(hd)


def test_autotune_and_tune_cache(tmp_path):
    import torch
    from paper_1812_02647_amd import hrms as H
    path = str(tmp_path / "tune.txt")
    x, offsets, _ = synth.batch(6, [300001, 1 << 18, 77777, 5, 4096, 123457], seed=29)
    xd, seen = to_device_input(x, "f32")
    h = make_handle(tune=path)
    try:
        for v in [0, 1, 2, 3]:
            case_log(f"autotune variant={NAMES[v]}")
            b = H.Batch1D(xd, offsets, v, 32)
            shape = H.hrms_autotune_1d(h, b.args, reps=2)
            assert len(shape) == 4 and all(s > 0 for s in shape[:2])
            torch.cuda.synchronize()
            out = fetch(b)
            for s in range(6):
                check_spectrum(b, out, seen, s, v, 32, check_f64=False, label="tuned")
            # a later run uses the tuned shape and still gives the oracle's bits
            out2 = fetch(b.run(h))
            for k in out:
                assert np.array_equal(out[k], out2[k], equal_nan=True)
        text = open(path).read().split()
        assert text[0] == "hrms-tune-v2" and text[1].startswith("gfx950")
    finally:
        H.hrms_destroy(h)
    # a corrupt cache is ignored
    with open(path, "w") as f:
        f.write("hrms-tune-v2 gfx950 256\n1 0 32 garbage\n")
    h = make_handle(tune=path)
    try:
        b = H.Batch1D(xd, offsets, 2, 32).run(h)
        torch.cuda.synchronize()
        check_spectrum(b, fetch(b), seen, 0, 2, 32, check_f64=False, label="corrupt-cache")
    finally:
        H.hrms_destroy(h)


def test_plan_query_reports_the_run_shape_and_launches(monkeypatch):
    """hrms_plan_1d names the shape a run uses and its harmonic-sum launches:
    two for eq. (2) on FP32 with a band at level 32 (that band runs in a
    launch of its own), one otherwise, and the forced shape when
    HRMS_FORCE_SHAPE names one; the query enqueues nothing."""
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets, _ = synth.batch(3, [1 << 17, 70001, 4096], seed=31)
    xd, _ = to_device_input(x, "f32")
    monkeypatch.delenv("HRMS_FORCE_SHAPE", raising=False)
    h = make_handle()
    try:
        case_log("plan query: default shapes")
        b = H.Batch1D(xd, offsets, 1, 32)
        b.max_snr.fill_(float("nan"))
        shape, n = H.hrms_plan_1d(h, b.args)
        assert shape[3] == 32 and n == 2
        torch.cuda.synchronize()
        assert torch.isnan(b.max_snr).all()          # nothing ran
        shape, n = H.hrms_plan_1d(h, H.Batch1D(xd, offsets, 1, 16).args)
        assert n == 1                                # no band at level 32
        for v in (0, 2, 3):
            shape, n = H.hrms_plan_1d(h, H.Batch1D(xd, offsets, v, 32).args)
            assert shape[3] == 0 and n == 1, (v, shape, n)
        case_log("plan query: forced shape")
        monkeypatch.setenv("HRMS_FORCE_SHAPE", "512:8:0:32")
        shape, n = H.hrms_plan_1d(h, H.Batch1D(xd, offsets, 2, 32).args)
        assert shape == (512, 8, 0, 32) and n == 2
    finally:
        H.hrms_destroy(h)


# every launch shape compiled into the library, forced in turn: wg:r:chunk:top
FUND_SHAPES = ["1024:8:16384:0", "1024:16:16384:0", "512:8:8192:0", "256:8:0:0", "256:8:0:32",
               "256:16:0:0", "512:8:0:0", "512:8:0:32"]
EQ1_SHAPES = ["256:8:0:0", "256:4:0:0", "512:8:0:0", "512:8:1:0"]


@pytest.mark.parametrize("variant,shape", [(v, s) for v in [1, 2, 3] for s in FUND_SHAPES] +
                         [(0, s) for s in EQ1_SHAPES])
def test_every_launch_shape_matches_oracle(monkeypatch, variant, shape):
    """Ragged batch (lengths from 3 to 2^18 + 3, Hmax 32 and 8) under each
    compiled shape, with and without the top-band split: the sampled outputs
    of every spectrum equal the oracle's bits."""
    import torch
    from paper_1812_02647_amd import hrms as H
    monkeypatch.setenv("HRMS_FORCE_SHAPE", shape)
    lengths = [(1 << 18) + 3, 3, 70001, 65536, 9999]
    hmax = np.array([32, 8, 32, 32, 16], np.uint8)
    x, offsets, _ = synth.batch(len(lengths), lengths, seed=37, comb_fraction=0.6)
    xd, seen = to_device_input(x, "f32")
    h = make_handle()
    try:
        case_log(f"forced shape {shape} variant={NAMES[variant]}")
        b = H.Batch1D(xd, offsets, variant, hmax).run(h)
        torch.cuda.synchronize()
        out = fetch(b)
        for s in range(len(lengths)):
            check_spectrum(b, out, seen, s, variant, int(hmax[s]), check_f64=False,
                           label=f"shape {shape}")
    finally:
        H.hrms_destroy(h)


@pytest.mark.parametrize("dtype", ["f16", "bf16", "f32"])
def test_eq1_lds_form_matches_oracle(monkeypatch, dtype):
    """eq. (1) in its LDS-staged form (shape 512:8:1) on 2-byte and FP32
    storage: spectra starting at every residue of the 16-byte vector, tiles
    ending mid-run, Hmax 1..32; every output equals the oracle's bits."""
    import torch
    from paper_1812_02647_amd import hrms as H
    monkeypatch.setenv("HRMS_FORCE_SHAPE", "512:8:1:0")
    lengths = [5001, 1, 7, 4099, 513, 12289, 2, 4096, 3]
    hmax = np.array([32, 1, 2, 4, 8, 16, 32, 32, 32], np.uint8)
    x, offsets, _ = synth.batch(len(lengths), lengths, seed=41, comb_fraction=0.5)
    xd, seen = to_device_input(x, dtype)
    h = make_handle()
    try:
        case_log(f"eq1 LDS form dtype={dtype}")
        b = H.Batch1D(xd, offsets, 0, hmax).run(h)
        torch.cuda.synchronize()
        out = fetch(b)
        for s in range(len(lengths)):
            check_spectrum(b, out, seen, s, 0, int(hmax[s]), idx=np.arange(lengths[s]),
                           check_f64=False, label=f"eq1 lds {dtype}")
    finally:
        H.hrms_destroy(h)


def _handle_with_env(**env):
    from paper_1812_02647_amd import hrms as H
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return H.hrms_create(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_injected_allocation_failure_leaves_handle_usable():
    """HRMS_FAULT_INJECT=alloc: the 1D, 2D and precision-form calls that need
    device memory fail with HRMS_E_NOMEM before enqueuing anything (outputs
    keep their fill); the entry point that allocates nothing still runs and
    matches the oracle; the handle is destroyed normally."""
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets, _ = synth.batch(3, [5000, 70001, 333], seed=23, comb_fraction=0.5)
    xd, seen = to_device_input(x, "f32")
    h = _handle_with_env(HRMS_FAULT_INJECT="alloc")
    try:
        case_log("fault injection: alloc")
        b = H.Batch1D(xd, offsets, H.HRMS_GREEDY, 16)
        b.max_snr.fill_(-3.0)
        torch.cuda.synchronize()
        with pytest.raises(H.HrmsError) as ei:
            b.run(h)
        assert ei.value.status == H.HRMS_E_NOMEM and "HRMS_FAULT_INJECT" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((b.max_snr == -3.0).all())
        # 2D plane and precision form
        a = H.hrms_run2d_args()
        a.nf, a.zmax, a.hmax, a.variant, a.ld, a.out_mask = 1000, 1, 8, H.HRMS_FREQBIN, 1000, 2
        plane = torch.ones(3 * 1000, dtype=torch.float32, device="cuda")
        st = torch.zeros(2, dtype=torch.float64, device="cuda")
        ms = torch.empty(3000, dtype=torch.float32, device="cuda")
        a.x, a.stats, a.max_snr = plane.data_ptr(), st.data_ptr(), ms.data_ptr()
        with pytest.raises(H.HrmsError) as ei:
            H.hrms_run_2d(h, a)
        assert ei.value.status == H.HRMS_E_NOMEM
        # the no-alloc entry point needs no allocation
        b.run_noalloc(h)
        torch.cuda.synchronize()
        out = fetch(b)
        for s in range(3):
            check_spectrum(b, out, seen, s, H.HRMS_GREEDY, 16, check_f64=False,
                           label="noalloc under alloc fault")
    finally:
        H.hrms_destroy(h)


@pytest.mark.parametrize("graphs", [True, False])
def test_injected_launch_failure_leaves_handle_destroyable(graphs):
    """HRMS_FAULT_INJECT=launch: every harmonic-sum launch reports
    HRMS_E_HIP (the statistics and constants before it run normally); the
    handle is destroyed normally and a new handle computes the same batch
    correctly."""
    import torch
    from paper_1812_02647_amd import hrms as H
    x, offsets, _ = synth.batch(2, [4099, 20000], seed=29, comb_fraction=0.5)
    xd, seen = to_device_input(x, "f32")
    env = {"HRMS_FAULT_INJECT": "launch"}
    if not graphs:
        env["HRMS_NO_GRAPH"] = "1"
    h = _handle_with_env(**env)
    try:
        case_log(f"fault injection: launch graphs={graphs}")
        b = H.Batch1D(xd, offsets, H.HRMS_MAX, 32)
        for _ in range(2):
            with pytest.raises(H.HrmsError) as ei:
                b.run(h)
            assert ei.value.status == H.HRMS_E_HIP
        with pytest.raises(H.HrmsError):
            b.run_noalloc(h)
        torch.cuda.synchronize()
    finally:
        H.hrms_destroy(h)
    h2 = H.hrms_create(0)
    try:
        b = H.Batch1D(xd, offsets, H.HRMS_MAX, 32).run(h2)
        torch.cuda.synchronize()
        out = fetch(b)
        for s in range(2):
            check_spectrum(b, out, seen, s, H.HRMS_MAX, 32, check_f64=False, label="after fault")
    finally:
        H.hrms_destroy(h2)
