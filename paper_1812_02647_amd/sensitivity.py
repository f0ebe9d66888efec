"""Sensitivity study of Sec. 3 (Figs. 1 and 2 of arXiv:1812.02647) on the device.

A simulated pulsar -- a modified von Mises pulse train in white Gaussian noise,
20 s sampled every 64 microseconds -- is Fourier transformed into a power
spectrum of 0.05 Hz bins, and every harmonic-sum variant is run over it with
Hmax = 32. The recovered SNR of a variant is the largest max-SNR output in a
small neighbourhood of where that variant places the pulsar:

  eq. (2)-(4): output n is a fundamental bin, so the bins floor(k) - 2 ..
               floor(k) + 2 around the pulsar's fractional bin k;
  eq. (1):     output n of level H is the H-th harmonic of fundamental n / H,
               so round(H k) - 2 .. round(H k) + 2 for every level H.

Two sets are studied (inputs from ``synth``): the response across one Fourier
bin (fundamental at k0 + delta for delta = 0, 1/8, ..., 7/8; Fig. 1) and the
response averaged over pulsar frequencies drawn across 2 .. 150 Hz (Fig. 2).
Everything runs through the C ABI of the library; there is no CPU path.

    python -m paper_1812_02647_amd.sensitivity      # prints one JSON object
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np

from . import hrms as H
from . import synth

VARIANT_NAMES = {H.HRMS_EQ1: "eq1", H.HRMS_MAX: "max", H.HRMS_FREQBIN: "freqbin",
                 H.HRMS_GREEDY: "greedy"}
HMAX = 32
HALF_WIDTH = 2   # neighbourhood half-width in output bins


def candidate_bins(kf: float, variant: int, n_bins: int, hmax: int = HMAX):
    """Output bins where a variant places a pulsar at fractional bin kf."""
    if variant == H.HRMS_EQ1:
        centres = [int(round(Hh * kf)) for Hh in (1 << l for l in range(int(math.log2(hmax)) + 1))]
    else:
        centres = [int(math.floor(kf))]
    out = set()
    for c in centres:
        out.update(range(c - HALF_WIDTH, c + HALF_WIDTH + 1))
    return np.array(sorted(b for b in out if 0 <= b < n_bins), np.int64)


def recovered(max_snr: np.ndarray, offsets: np.ndarray, meta, variant: int,
              hmax: int = HMAX) -> np.ndarray:
    """Recovered SNR of each spectrum of a packed batch."""
    out = np.empty(len(meta), np.float64)
    for s, (kf, _, _) in enumerate(meta):
        n = int(offsets[s + 1] - offsets[s])
        b = candidate_bins(kf, variant, n, hmax)
        out[s] = float(max_snr[offsets[s] + b].max())
    return out


def run_variants(handle, x: np.ndarray, offsets: np.ndarray, meta, hmax: int = HMAX,
                 variants=(H.HRMS_EQ1, H.HRMS_MAX, H.HRMS_FREQBIN, H.HRMS_GREEDY)):
    """Recovered SNR per variant over a packed batch, statistics computed on
    the device per spectrum."""
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to("cuda")
    res = {}
    for v in variants:
        b = H.Batch1D(xd, offsets, v, hmax, out_mask=H.HRMS_OUT_MAXSNR, want_consts=False)
        b.run(handle)
        torch.cuda.synchronize()
        res[v] = recovered(b.max_snr.cpu().numpy(), offsets, meta, v, hmax)
    return res


def summarise(bin_res, bin_meta, sweep_res) -> dict:
    deltas = sorted({d for _, d, _ in bin_meta})
    dl = np.array([d for _, d, _ in bin_meta])
    out = {"deltas": deltas, "per_delta": {}, "averaged": {}, "averaged_vs_eq1": {},
           "offbin_vs_onbin": {}}
    for v, r in bin_res.items():
        name = VARIANT_NAMES[v]
        per = [float(r[dl == d].mean()) for d in deltas]
        out["per_delta"][name] = [round(p, 3) for p in per]
        out["offbin_vs_onbin"][name] = round(per[deltas.index(0.5)] / per[0], 4)
    for v, r in sweep_res.items():
        out["averaged"][VARIANT_NAMES[v]] = round(float(r.mean()), 3)
    ref = out["averaged"]["eq1"]
    for k, a in out["averaged"].items():
        out["averaged_vs_eq1"][k] = round(a / ref, 4)
    return out


def main() -> int:
    handle = H.hrms_create(0)
    try:
        xb, ob, mb = synth.sensitivity_set()
        xs, os_, ms = synth.frequency_sweep_set()
        res = summarise(run_variants(handle, xb, ob, mb), mb, run_variants(handle, xs, os_, ms))
    finally:
        H.hrms_destroy(handle)
    res["setup"] = {"samples": synth.OBS_SAMPLES, "sample_s": synth.SAMPLE_SECONDS,
                    "bin_hz": 1.0 / synth.OBS_SECONDS, "hmax": HMAX, "profile": "von Mises kappa=20",
                    "amplitude": 0.1, "bin_set": "k0 in {150, 400}, 3 noise draws per delta",
                    "sweep_set": "32 pulsars, 2..150 Hz"}
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
