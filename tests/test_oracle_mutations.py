"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of the oracle source (a wrong
rounding direction, an off-by-one window, a dropped term, a wrong constant, a
reversed tie rule ...), builds it with gcc into a temporary directory, routes
the oracle front end to it and runs the pin tests. At least one pin must fail
for every mistake. Nothing here touches the GPU or the library under test.
"""
import inspect
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "hrms_oracle.c")

# (name, text in the source, replacement)
MUTATIONS = [
    ("eq1 rounds down", "return (2 * a + b) / (2 * b);", "return a / b;"),
    ("eq1 rounds half down", "return (2 * a + b) / (2 * b);", "return (2 * a + b - 1) / (2 * b);"),
    ("max window starts one bin late", "double m = x[(int64_t)i * n];",
     "double m = x[(int64_t)i * n + 1];"),
    ("max window drops its last bin", "for (int j = 1; j < i; ++j) {",
     "for (int j = 1; j < i - 1; ++j) {"),
    ("freqbin reads (i-1) n", "acc = rnd(f32, acc + x[(int64_t)i * n]);",
     "acc = rnd(f32, acc + x[(int64_t)(i - 1) * n + (i == 1 ? n : 0)]);"),
    ("freqbin drops the fundamental", "for (int i = 1; i <= H; ++i) acc = rnd(f32, acc + x[(int64_t)i * n]);",
     "for (int i = 2; i <= H; ++i) acc = rnd(f32, acc + x[(int64_t)i * n]);"),
    ("greedy takes ties to the right", "        if (b > a) {\n            acc = rnd(f32, acc + b);\n            j += 1;\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path",
     "        if (b >= a) {\n            acc = rnd(f32, acc + b);\n            j += 1;\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path"),
    ("greedy never moves", "            acc = rnd(f32, acc + b);\n            j += 1;\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path",
     "            acc = rnd(f32, acc + b);\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path"),
    ("greedy reads harmonic k-1", "        double a = x[(int64_t)k * n + j];\n        double b = x[(int64_t)k * n + j + 1];\n        if (b > a) {\n            acc = rnd(f32, acc + b);\n            j += 1;\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path",
     "        double a = x[(int64_t)(k - 1) * n + j];\n        double b = x[(int64_t)(k - 1) * n + j + 1];\n        if (b > a) {\n            acc = rnd(f32, acc + b);\n            j += 1;\n        } else {\n            acc = rnd(f32, acc + a);\n        }\n    }\n    return acc;\n}\n\n/*\n * Exhaustive-path"),
    ("level domain one too long", "return n < N / H;", "return n <= N / H;"),
    ("scale 1/H instead of 1/sqrt(H)", "return rnd(f32, 1.0 / sqrt((double)H));",
     "return rnd(f32, 1.0 / (double)H);"),
    ("sample instead of population sigma", "long double v = s2 / (long double)n - m * m;",
     "long double v = (s2 - (long double)n * m * m) / (long double)(n - 1);"),
    ("max psi uses 1/i", "psi = psi + 1.0 / ((double)i * (double)i);", "psi = psi + 1.0 / (double)i;"),
    ("max mean drops the -1", "sum_mean = sum_mean + (mu + sigma * (hn - 1.0));",
     "sum_mean = sum_mean + (mu + sigma * hn);"),
    ("greedy variance 1.5", "var_s = (sigma * sigma) * (1.0 + 1.25 * (double)(H - 1));",
     "var_s = (sigma * sigma) * (1.0 + 1.5 * (double)(H - 1));"),
    ("greedy mean sigma instead of sigma/2", "mean_s = mu + (double)(H - 1) * (mu + 0.5 * sigma);",
     "mean_s = mu + (double)(H - 1) * (mu + sigma);"),
    ("freqbin variance H^2", "var_s = (double)H * (sigma * sigma);",
     "var_s = (double)H * (double)H * (sigma * sigma);"),
    ("snr adds the mean", "static double snr_of(double h, double m, double q, int f32) { return rnd(f32, rnd(f32, h - m) * q); }",
     "static double snr_of(double h, double m, double q, int f32) { return rnd(f32, rnd(f32, h + m) * q); }"),
    ("best level ties move up", "                if (l == 0 || snr > best) {\n                    best = snr;\n                    best_level = H;\n                }\n            }\n        }\n        if (max_snr) max_snr[k] = best;\n        if (best_h) best_h[k] = (uint8_t)best_level;\n    }\n    return OE_OK;\n}\n\n/* ----",
     "                if (l == 0 || snr >= best) {\n                    best = snr;\n                    best_level = H;\n                }\n            }\n        }\n        if (max_snr) max_snr[k] = best;\n        if (best_h) best_h[k] = (uint8_t)best_level;\n    }\n    return OE_OK;\n}\n\n/* ----"),
    ("f32 mode skips rounding of sums", "static double rnd(int f32, double v) { return f32 ? (double)(float)v : v; }",
     "static double rnd(int f32, double v) { (void)f32; return v; }"),
    ("2d rows round half up", "return a >= 0 ? round_half_up(a, b) : -round_half_up(-a, b);",
     "return a >= 0 ? round_half_up(a, b) : -((-(2 * a + b) + 2 * b - 1) / (2 * b));"),
    ("2d greedy never moves", "                acc = rnd(f32, acc + b);\n                j += 1;",
     "                acc = rnd(f32, acc + b);"),
    ("2d freqbin uses the level-1 row", "int64_t row = round_half_away((int64_t)i * z, H) + zmax;\n            acc = rnd(f32, acc + x[row * ld + (int64_t)i * mbin]);",
     "int64_t row = round_half_away((int64_t)z, 1) + zmax;\n            acc = rnd(f32, acc + x[row * ld + (int64_t)i * mbin]);"),
    ("2d rows truncate toward zero", "return a >= 0 ? round_half_up(a, b) : -round_half_up(-a, b);",
     "return a / b;"),
    ("2d eq1 frequency rounds down", "acc = rnd(f32, acc + x[row * ld + round_half_up((int64_t)i * mbin, H)]);",
     "acc = rnd(f32, acc + x[row * ld + (int64_t)i * mbin / H]);"),
    ("2d max window drops its last bin", "for (int j = 1; j < i; ++j)\n                if (w[j] > m)",
     "for (int j = 1; j < i - 1; ++j)\n                if (w[j] > m)"),
    ("2d max reads the fundamental's row", "            const double* w = x + row * ld + (int64_t)i * mbin;",
     "            const double* w = x + (round_half_away((int64_t)z, H) + zmax) * ld + (int64_t)i * mbin;"),
    ("opt recurrence never steps right", "m = P[j - 1] > P[j] ? P[j - 1] : P[j];", "m = P[j];"),
    ("opt recurrence keeps the last state", "    double best = P[0];\n    for (int j = 1; j < H; ++j)\n        if (P[j] > best) best = P[j];",
     "    double best = P[H - 1];"),
    ("opt paths may step by two", "            j += (path >> (k - 2)) & 1;", "            j += 2 * ((path >> (k - 2)) & 1);"),
    ("opt paths skip the last harmonic", "        for (int k = 2; k <= H; ++k) {\n            j += (path >> (k - 2)) & 1;",
     "        for (int k = 2; k < H; ++k) {\n            j += (path >> (k - 2)) & 1;"),
    ("scale uses binary64 1/mu", "double inv = (double)(float)(1.0 / mu);", "double inv = 1.0 / mu;"),
    ("2d fdot-drift Greedy drifts toward zero", "const int64_t s = z > 0 ? 1 : (z < 0 ? -1 : 0);",
     "const int64_t s = z > 0 ? -1 : (z < 0 ? 1 : 0);"),
    ("2d fdot-drift Greedy never drifts in fdot", "        if (pick & 2) d += s;\n", ""),
    ("2d fdot-drift Greedy never steps in frequency", "        if (pick & 1) j += 1;\n", ""),
    ("2d fdot-drift Greedy takes ties to the later candidate",
     "            if (cand[t] > cand[pick]) pick = t;", "            if (cand[t] >= cand[pick]) pick = t;"),
    ("2d fdot-drift Greedy clamps one row short at the top",
     "return r < -zmax ? -zmax : (r > zmax ? zmax : r);",
     "return r < -zmax ? -zmax : (r > zmax - 1 ? zmax - 1 : r);"),
    ("2d fdot-drift Greedy reads the row of harmonic k-1",
     "const int64_t rk = round_half_away((int64_t)k * z, H);",
     "const int64_t rk = round_half_away((int64_t)(k - 1) * z, H);"),
    ("2d fdot-drift Greedy z = 0 row takes the drifting constants",
     "int c = (variant == OV_GREEDY_FZ && z == 0) ? nl + l : l;", "int c = l;"),
    ("2d fdot-drift Greedy mean of a max of four as of two",
     "mean_s = mu + (double)(H - 1) * (mu + (13.0 / 12.0) * sigma);",
     "mean_s = mu + (double)(H - 1) * (mu + 0.5 * sigma);"),
    ("2d fdot-drift Greedy variance of a max of four as of two",
     "var_s = (sigma * sigma) * (1.0 + (205.0 / 144.0) * (double)(H - 1));",
     "var_s = (sigma * sigma) * (1.0 + 1.25 * (double)(H - 1));"),
]


def _pin_cases():
    """Every pin test with each of its parameter sets, as zero-argument calls."""
    cases = []
    for name, fn in inspect.getmembers(P, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        combos = [{}]
        for m in params:
            argnames = [a.strip() for a in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
            new = []
            for c in combos:
                for val in m.args[1]:
                    vals = val if len(argnames) > 1 else (val,)
                    d = dict(c)
                    d.update(zip(argnames, vals))
                    new.append(d)
            combos = new
        for c in combos:
            cases.append((name, fn, c))
    return cases


def _build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    # the first occurrence is the one meant (the 1D driver precedes the 2D one)
    assert src.count(old) >= 1, f"mutation target not present: {old[:60]!r}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", *O.CFLAGS, "-o", str(so), str(mpath), "-lm"])
    return str(so)


def test_pins_pass_on_the_real_oracle():
    for name, fn, kw in _pin_cases():
        fn(**kw)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    so = _build_mutant(tmp_path, old, new)
    caught = []
    with O.use_library(so):
        for tname, fn, kw in _pin_cases():
            try:
                fn(**kw)
            except (AssertionError, ValueError):
                caught.append(tname)
                break
    assert caught, f"no pin fails when the oracle has the mistake: {name}"
