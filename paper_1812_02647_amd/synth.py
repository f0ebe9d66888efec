"""Seeded synthetic inputs: exponential (chi-square, 2 dof) power spectra and
f-fdot planes with injected harmonic combs.

This module only draws inputs. It holds none of the harmonic-sum arithmetic
and is the one piece shared by the device path's callers and the CPU oracle's
callers, so both see byte-identical inputs.

Workload recipes (sizes, value distributions, comb structure) follow the
simulation set-up of arXiv:1812.02647, Sec. 3: noise-only power spectra plus an
artificial periodic signal whose power is spread over harmonics. No dataset is
involved.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_LIB = os.path.join(_HERE, "libhrms_synth.so")

SEED_BASE = 1812026470


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.synth_exponential_f32.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64,
                                            C.c_void_p, C.c_int]
        L.synth_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.synth_uniform.restype = C.c_double
        L.synth_u64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.synth_u64.restype = C.c_uint64
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def exponential(seed: int, stream: int, count: int, start: int = 0, out=None, threads=None):
    """``count`` Exp(1) bins of stream ``stream`` starting at draw ``start``."""
    if out is None:
        out = np.empty(count, np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.size == count
    rc = lib().synth_exponential_f32(seed, stream, start, count,
                                     out.ctypes.data_as(C.c_void_p),
                                     threads or default_threads())
    if rc != 0:
        raise RuntimeError("synth_exponential_f32 failed")
    return out


def sinc2(d: float) -> float:
    if d == 0.0:
        return 1.0
    s = math.sin(math.pi * d) / (math.pi * d)
    return s * s


def inject_integer_comb(x, f0: int, amps):
    """Harmonic i (1-based) of an on-bin signal adds amps[i-1] at bin i*f0."""
    for i, a in enumerate(amps, start=1):
        k = i * f0
        if k < x.size:
            x[k] = np.float32(x[k] + np.float32(a))
    return x


def inject_fractional_comb(x, f0: float, amps):
    """Harmonic i at frequency i*f0 (in bins): the unwindowed DFT of a pure tone
    puts A*sinc^2(d) in the bin below and A*sinc^2(1-d) in the bin above, with
    d the fractional part of i*f0."""
    for i, a in enumerate(amps, start=1):
        f = i * f0
        k = int(math.floor(f))
        d = f - k
        if k < x.size:
            x[k] = np.float32(x[k] + np.float32(a * sinc2(d)))
        if k + 1 < x.size:
            x[k + 1] = np.float32(x[k + 1] + np.float32(a * sinc2(1.0 - d)))
    return x


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_spectrum(n: int = 65536, seed: int = SEED_BASE, f0: int = 1000, harmonics: int = 8,
                    amp: float = 20.0):
    """One FP32 spectrum of Exp(1) noise plus an on-bin comb at fundamental bin
    ``f0`` whose harmonic i has amplitude amp/i."""
    x = exponential(seed, 0, n)
    if harmonics:
        inject_integer_comb(x, f0, [amp / i for i in range(1, harmonics + 1)])
    return x


def batch(n_spectra: int, n_bins, seed: int = SEED_BASE + 1, comb_fraction: float = 0.01,
          harmonics: int = 16, amp: float = 5.0, f0_range=(100.0, 50000.0), out=None,
          threads=None):
    """Packed batch of spectra (DM trials). ``n_bins`` is an int (equal lengths)
    or a sequence of lengths. A fraction of the trials carries a comb at a
    random fractional fundamental with amplitudes amp/sqrt(i).

    Returns ``(x, offsets, combs)``; ``combs`` lists (spectrum, f0).
    """
    if np.isscalar(n_bins):
        lengths = np.full(n_spectra, int(n_bins), np.int64)
    else:
        lengths = np.asarray(n_bins, np.int64)
        assert lengths.size == n_spectra
    offsets = np.zeros(n_spectra + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    if out is None:
        out = np.empty(total, np.float32)
    assert out.size >= total
    for s in range(n_spectra):
        exponential(seed, s, int(lengths[s]), out=out[offsets[s]:offsets[s + 1]],
                    threads=threads)
    rng = np.random.default_rng(seed)
    n_comb = int(round(comb_fraction * n_spectra))
    chosen = np.sort(rng.choice(n_spectra, size=n_comb, replace=False)) if n_comb else []
    combs = []
    amps = [amp / math.sqrt(i) for i in range(1, harmonics + 1)]
    for s in chosen:
        n = int(lengths[s])
        hi = min(f0_range[1], n / harmonics)
        lo = min(f0_range[0], hi / 2)
        f0 = float(rng.uniform(lo, hi))
        inject_fractional_comb(out[offsets[s]:offsets[s + 1]], f0, amps)
        combs.append((int(s), f0))
    return out[:total], offsets, combs


def uneven_lengths(n_spectra: int = 512, seed: int = SEED_BASE + 3, lo_exp: int = 14,
                   hi_exp: int = 23):
    """Lengths drawn log-uniform in [2^lo_exp, 2^hi_exp) and Hmax drawn uniformly
    from {8, 16, 32}, one pair per spectrum."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, n_spectra)
    lengths = np.floor(2.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    hmax = rng.choice(np.array([8, 16, 32], np.uint8), size=n_spectra)
    return lengths, hmax


def plane(nf: int = 1 << 21, zmax: int = 42, seed: int = SEED_BASE + 2, n_comb: int = 20,
          harmonics: int = 8, amp: float = 20.0, f0_max=None, z0_max: int = 5, threads=None):
    """f-fdot plane of shape (2*zmax+1, nf), row r holding fdot z = r - zmax.

    ``n_comb`` accelerated combs are injected, half on-bin and half at a
    fractional fundamental, harmonic i at (i*f0, i*z0) with amplitude amp/i and
    integer z0 in [-z0_max, z0_max]. Returns ``(x2d, combs)`` with combs a list
    of (f0, z0).
    """
    rows = 2 * zmax + 1
    x = np.empty((rows, nf), np.float32)
    for r in range(rows):
        exponential(seed, r, nf, out=x[r], threads=threads)
    rng = np.random.default_rng(seed)
    if f0_max is None:
        f0_max = nf / (2 * harmonics)
    combs = []
    amps = [amp / i for i in range(1, harmonics + 1)]
    for c in range(n_comb):
        z0 = int(rng.integers(-z0_max, z0_max + 1))
        if c < n_comb // 2:
            f0 = float(int(rng.integers(max(1, min(100, f0_max // 2)), f0_max)))
        else:
            f0 = float(rng.uniform(min(100.0, f0_max / 2), f0_max))
        for i, a in enumerate(amps, start=1):
            zr = i * z0 + zmax
            if not (0 <= zr < rows):
                continue
            f = i * f0
            k = int(math.floor(f))
            d = f - k
            if k < nf:
                x[zr, k] = np.float32(x[zr, k] + np.float32(a * sinc2(d)))
            if d > 0.0 and k + 1 < nf:
                x[zr, k + 1] = np.float32(x[zr, k + 1] + np.float32(a * sinc2(1.0 - d)))
        combs.append((f0, z0))
    return x, combs


# ---------------------------------------------------------------------------
# Simulated pulsar observation (Sec. 3)
# ---------------------------------------------------------------------------

# 20 s of data sampled every 64 microseconds: 312500 samples, so the power
# spectrum has 156251 bins of width 1 / 20 s = 0.05 Hz.
OBS_SECONDS = 20.0
SAMPLE_SECONDS = 64e-6
OBS_SAMPLES = 312500


def pulsar_time_series(f0_hz: float, amp: float, kappa: float = 20.0, phase: float = 0.0,
                       seed: int = SEED_BASE + 4, n: int = OBS_SAMPLES,
                       ts: float = SAMPLE_SECONDS):
    """Pulse train with a modified von Mises profile exp(kappa (cos(2 pi phi) - 1))
    (unit peak, duty cycle shrinking with kappa) at frequency f0_hz and peak
    amplitude amp, plus white Gaussian noise of unit variance (numpy's PCG64
    generator seeded with ``seed``). Binary64."""
    t = np.arange(n, dtype=np.float64) * ts
    prof = np.exp(kappa * (np.cos(2.0 * np.pi * (f0_hz * t + phase)) - 1.0))
    return amp * prof + np.random.default_rng(seed).standard_normal(n)


def pulsar_power_spectrum(f0_hz: float, amp: float, kappa: float = 20.0, phase: float = 0.0,
                          seed: int = SEED_BASE + 4, n: int = OBS_SAMPLES,
                          ts: float = SAMPLE_SECONDS):
    """FP32 power spectrum |X_k|^2 / n, k = 0 .. n/2, of the mean-removed pulsar
    time series (numpy's real FFT in binary64, then rounded once). Noise bins
    are exponential with unit mean; the DC bin is zero."""
    x = pulsar_time_series(f0_hz, amp, kappa, phase, seed, n, ts)
    x = x - x.mean()
    X = np.fft.rfft(x)
    return ((X.real * X.real + X.imag * X.imag) / n).astype(np.float32)


def sensitivity_set(k0_list=(150, 400), deltas=tuple(np.arange(8) / 8.0), seeds: int = 3,
                    amp: float = 0.1, kappa: float = 20.0, seed: int = SEED_BASE + 4):
    """Spectra for the response across one Fourier bin: pulsars at
    f0 = (k0 + delta) * 0.05 Hz for every k0, delta and noise draw. Returns
    ``(x, offsets, meta)``: the packed FP32 spectra and, per spectrum,
    (k0 + delta, delta, draw)."""
    df = 1.0 / OBS_SECONDS
    spectra, meta = [], []
    for d in deltas:
        for k0 in k0_list:
            for r in range(seeds):
                kf = k0 + float(d)
                s = seed + 7919 * k0 + 104729 * int(round(float(d) * 1024)) + r
                spectra.append(pulsar_power_spectrum(kf * df, amp, kappa, 0.0, s))
                meta.append((kf, float(d), r))
    offsets = np.zeros(len(spectra) + 1, np.int64)
    np.cumsum([s.size for s in spectra], out=offsets[1:])
    return np.concatenate(spectra), offsets, meta


def frequency_sweep_set(n_freq: int = 32, lo_hz: float = 2.0, hi_hz: float = 150.0,
                        amp: float = 0.1, kappa: float = 20.0, seed: int = SEED_BASE + 5):
    """Spectra for the averaged response: n_freq pulsars at frequencies drawn
    uniformly in [lo_hz, hi_hz) (any fractional bin offset), one noise draw
    each. Returns ``(x, offsets, meta)`` with meta[k] = (f0 / 0.05 Hz, frac, 0)."""
    df = 1.0 / OBS_SECONDS
    rng = np.random.default_rng(seed)
    f0s = rng.uniform(lo_hz, hi_hz, n_freq)
    spectra, meta = [], []
    for k, f0 in enumerate(f0s):
        spectra.append(pulsar_power_spectrum(float(f0), amp, kappa, 0.0, seed + 1 + k))
        kf = float(f0) / df
        meta.append((kf, kf - math.floor(kf), 0))
    offsets = np.zeros(len(spectra) + 1, np.int64)
    np.cumsum([s.size for s in spectra], out=offsets[1:])
    return np.concatenate(spectra), offsets, meta
