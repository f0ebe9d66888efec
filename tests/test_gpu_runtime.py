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


# every launch shape compiled into the library, forced in turn: wg:r:chunk:top
FUND_SHAPES = ["1024:8:16384:0", "1024:16:16384:0", "512:8:8192:0", "256:8:0:0", "256:8:0:32",
               "256:16:0:0", "512:8:0:0", "512:8:0:32"]
EQ1_SHAPES = ["256:8:0:0", "256:4:0:0", "512:8:0:0"]


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
