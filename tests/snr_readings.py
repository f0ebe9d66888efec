"""Readings of the SNR that Sec. 3 reports without defining, applied to the
oracle's binary64 sums of the simulated pulsar (test infrastructure).

The library standardises each level against the exact null moments of the
variant (m_H, 1/q_H; "standardised" below). The alternatives a reader of
Sec. 3 could take instead:

  raw          the sum h_H itself, no standardisation;
  naive        (h_H - sqrt(H) mu) / sigma for every variant: the null moments of
               eq. (1) and freq-bin, ignoring that Max and Greedy take maxima;
  empirical    (h_H - mean) / std with the mean and standard deviation of the
               level's outputs over the spectrum (signal included);
  robust       (h_H - median) / (1.4826 MAD) over the level's outputs.

For every reading the recovered SNR of a pulsar is the largest per-bin maximum
over the levels, taken over the outputs where the variant places the pulsar
(fundamental bins floor(k) - 2 .. floor(k) + 2 for eq. (2)-(4); for eq. (1)
the bins round(H k) - 2 .. round(H k) + 2 of every level H).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import oracle as O

HMAX = 32
READINGS = ("standardised", "raw", "naive", "empirical", "robust")
VARIANTS = (O.EQ1, O.MAX, O.FREQBIN, O.GREEDY)


def _levels_snr(h, variant, mu, sd, reading, N):
    """Per-level SNR planes (NaN where a level does not exist)."""
    nl = h.shape[0]
    out = np.full_like(h, np.nan)
    _, _, m64, q64 = O.snr_consts(variant, mu, sd, HMAX)
    for l in range(nl):
        H = 1 << l
        ln = N if variant == O.EQ1 else N >> l
        v = h[l, :ln]
        if reading == "standardised":
            s = (v - m64[l]) * q64[l]
        elif reading == "raw":
            s = v.copy()
        elif reading == "naive":
            s = (v - math.sqrt(H) * mu) / sd
        elif reading == "empirical":
            s = (v - np.nanmean(v)) / np.nanstd(v)
        elif reading == "robust":
            med = np.nanmedian(v)
            s = (v - med) / (1.4826 * np.nanmedian(np.abs(v - med)))
        else:
            raise ValueError(reading)
        out[l, :ln] = s
    return out


def near(kf, variant, N):
    """Per level, the outputs where the variant places a pulsar at bin kf."""
    nl = O.num_levels(HMAX)
    res = []
    for l in range(nl):
        c = int(round((1 << l) * kf)) if variant == O.EQ1 else int(math.floor(kf))
        res.append([b for b in range(c - 2, c + 3) if 0 <= b < N])
    return res


def max_literal_window(xs):
    """Level planes of Max with eq. (2)'s window taken as printed,
    x(i n + 1) .. x(i n + i), in binary64 (numpy; outputs past the last full
    window are NaN)."""
    N = xs.size
    nl = O.num_levels(HMAX)
    h = np.full((nl, N), np.nan)
    acc = np.zeros(N)
    valid = np.ones(N, bool)
    n = np.arange(N)
    for i in range(1, HMAX + 1):
        ok = i * n + i < N
        t = np.full(N, np.nan)
        m = n[ok]
        t[ok] = np.max(np.stack([xs[i * m + j] for j in range(1, i + 1)]), axis=0)
        acc = acc + t
        valid &= ok
        if i & (i - 1) == 0:
            l = i.bit_length() - 1
            h[l] = np.where(valid, acc / math.sqrt(i), np.nan)
    return h


def recovered(xs, kf, literal_max=False):
    """{reading: [recovered SNR per variant]} for one spectrum (with
    literal_max, Max's window as printed instead of the adopted one)."""
    xs = np.asarray(xs, np.float64)
    N = xs.size
    mu, sd = O.stats(xs)
    out = {r: [] for r in READINGS}
    for v in VARIANTS:
        if v == O.MAX and literal_max:
            h = max_literal_window(xs)
        else:
            h, _, _, _ = O.hrms_1d(xs, v, HMAX, f32=False, want_snr=False)
        bins = near(kf, v, N)
        for r in READINGS:
            snr = _levels_snr(h, v, mu, sd, r, N)
            if v == O.MAX and literal_max:
                snr[np.isnan(h)] = np.nan
            best = -np.inf
            for l, bl in enumerate(bins):
                for b in bl:
                    if not np.isnan(snr[l, b]):
                        best = max(best, snr[l, b])
            out[r].append(best)
    return out


def study(x, offsets, meta, threads=8, literal_max=False):
    """{reading: array [spectrum, variant]} over a packed set of spectra."""
    def one(s):
        return recovered(x[offsets[s]:offsets[s + 1]], meta[s][0], literal_max)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        rows = list(ex.map(one, range(len(meta))))
    return {r: np.array([row[r] for row in rows]) for r in READINGS}


def claims(bin_res, deltas, sweep_res):
    """The four prose claims of Sec. 3 as numbers, per reading:
    freq-bin's off-bin (delta 1/2) over on-bin recovery, Max's off-bin over
    on-bin recovery and its flatness (smallest over largest mean across the
    bin offsets), and each variant's averaged recovery over eq. (1)'s."""
    table = {}
    ds = sorted(set(deltas))
    for r in READINGS:
        b = bin_res[r]
        per = np.array([[b[deltas == d, v].mean() for d in ds] for v in range(4)])
        avg = sweep_res[r].mean(axis=0)
        table[r] = {
            "freqbin_off_over_on": float(per[2, ds.index(0.5)] / per[2, 0]),
            "max_off_over_on": float(per[1, ds.index(0.5)] / per[1, 0]),
            "max_flatness": float(per[1].min() / per[1].max()),
            "avg_over_eq1": {n: float(avg[v] / avg[0]) for v, n in
                             enumerate(("eq1", "max", "freqbin", "greedy"))},
            "best_delta_is_centre": [int(np.argmax(per[v])) == 0 for v in range(4)],
        }
    return table
