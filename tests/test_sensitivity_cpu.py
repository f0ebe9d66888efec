"""The sensitivity claims of Sec. 3 (Figs. 1 and 2 of arXiv:1812.02647), checked
on the oracle over the simulated pulsar of that section.

The figures themselves are not available, so the prose claims are checked:
  - the highest SNR is recovered when the pulsar sits on a Fourier bin centre
    (Fig. 1 discussion; strictly for eq. (1) and freq-bin, within the spread of
    the noise draws for Max and Greedy, whose responses are flatter there);
  - freq-bin loses more than half of its SNR between bin centres (Fig. 1);
  - averaged over pulsar frequencies, Greedy recovers about what the standard
    sum does and freq-bin about 20% less (Fig. 2).
The paper also reports an averaged loss of about 40% for Max and a response
flat across the bin. With the SNR read here as a standardisation against the
exact null moments of each variant (the Max null includes the bias of taking
maxima), Max loses far less and is not flat. The last two tests hold the
adopted reading to the figures it gives and show that no other reading of the
SNR (raw sums, eq. (1)'s null for every variant, empirical or robust moments
of each level), nor Max's window taken as printed, reaches the Max claims.

The recovered SNR is the largest max-SNR output near where a variant places the
pulsar (fundamental bins around floor(k) for eq. (2)-(4); round(H k) for every
level H of eq. (1)).
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_1812_02647_amd import synth

HMAX = 32


def near(kf, variant, n):
    if variant == O.EQ1:
        cs = [int(round(H * kf)) for H in O.levels(HMAX)]
    else:
        cs = [int(math.floor(kf))]
    return sorted({b for c in cs for b in range(c - 2, c + 3) if 0 <= b < n})


def oracle_recovered(x, offsets, meta):
    def one(s):
        xs = x[offsets[s]:offsets[s + 1]].astype(np.float64)
        mu, sd = O.stats(xs)
        row = []
        for v in (O.EQ1, O.MAX, O.FREQBIN, O.GREEDY):
            _, ms, _, _ = O.hrms_1d(xs, v, HMAX, f32=True, mu=mu, sigma=sd)
            row.append(max(ms[b] for b in near(meta[s][0], v, xs.size)))
        return row

    with ThreadPoolExecutor(max_workers=8) as ex:
        rows = list(ex.map(one, range(len(meta))))
    return np.array(rows)   # [spectrum, variant]


@pytest.fixture(scope="module")
def bin_study():
    x, offsets, meta = synth.sensitivity_set()
    return oracle_recovered(x, offsets, meta), np.array([m[1] for m in meta])


@pytest.fixture(scope="module")
def sweep_study():
    x, offsets, meta = synth.frequency_sweep_set()
    return oracle_recovered(x, offsets, meta)


def test_bin_centre_response(bin_study):
    r, d = bin_study
    deltas = sorted(set(d))
    for v in range(4):
        per = [r[d == dd, v].mean() for dd in deltas]
        # the centre is (within the spread of 6 noise draws) the best place,
        # and mid-bin is worse than the centre for every variant
        assert per[0] >= 0.97 * max(per), (v, per)
        assert per[deltas.index(0.5)] < per[0], (v, per)
        if v in (O.EQ1, O.FREQBIN):
            assert int(np.argmax(per)) == 0, (v, per)


def test_freqbin_loses_over_half_between_bins(bin_study):
    r, d = bin_study
    on, off = r[d == 0.0, 2].mean(), r[d == 0.5, 2].mean()
    assert off < 0.5 * on, (on, off)
    # eq. (1) and Greedy follow the drifting harmonics and keep most of it
    for v in (0, 3):
        assert r[d == 0.5, v].mean() > 0.6 * r[d == 0.0, v].mean()


def test_averaged_losses(sweep_study):
    avg = sweep_study.mean(axis=0)
    eq1, mx, fb, gr = avg
    assert 0.70 <= fb / eq1 <= 0.90, avg          # "about 20%" lower
    assert abs(gr / eq1 - 1.0) <= 0.15, avg       # Greedy similar to standard
    assert mx < eq1, avg


# --------------------------------------------------------------------------
# The SNR that Sec. 3 reports is not defined there. Every plausible reading
# (tests/snr_readings.py) is applied to the same sums; the adopted one
# (standardisation against the exact null of each variant) is held to the
# figures it gives, and no reading -- nor Max's window taken as printed --
# gives Max the averaged loss of about 40% or a response flat across the bin
# that the paper reports, so that gap is a property of the paper's unstated
# set-up, not of the reading taken here.
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def readings():
    from tests import snr_readings as R
    xb, ob, mb = synth.sensitivity_set()
    xs, os_, ms = synth.frequency_sweep_set()
    d = np.array([m[1] for m in mb])
    adopted = R.claims(R.study(xb, ob, mb), d, R.study(xs, os_, ms))
    literal = R.claims(R.study(xb, ob, mb, literal_max=True), d,
                       R.study(xs, os_, ms, literal_max=True))
    return adopted, literal


def test_adopted_snr_reading_measured_figures(readings):
    s = readings[0]["standardised"]
    assert 0.28 <= s["freqbin_off_over_on"] <= 0.36, s     # measured 0.318
    assert 0.70 <= s["max_off_over_on"] <= 0.77, s          # measured 0.734
    assert 0.52 <= s["max_flatness"] <= 0.60, s             # measured 0.556
    assert 0.88 <= s["avg_over_eq1"]["max"] <= 0.94, s      # measured 0.911
    assert 0.83 <= s["avg_over_eq1"]["freqbin"] <= 0.89, s  # measured 0.858
    assert 0.90 <= s["avg_over_eq1"]["greedy"] <= 0.95, s   # measured 0.927


def test_no_snr_reading_gives_max_a_forty_percent_loss(readings):
    for table in readings:
        for name, r in table.items():
            assert r["avg_over_eq1"]["max"] > 0.85, (name, r)
            assert r["max_flatness"] < 0.80, (name, r)
            # freq-bin's off-bin loss of more than half holds under every reading
            assert r["freqbin_off_over_on"] < 0.5, (name, r)
