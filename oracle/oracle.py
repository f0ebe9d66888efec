"""ctypes front end of the CPU oracle (``hrms_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library under test. It shares
no code with the HIP implementation; inputs reach it as numpy arrays.

Every routine follows the definitions of arXiv:1812.02647: eq. (1) (Sec. 1) and
eq. (2)-(4) (Sec. 2). See ``hrms_oracle.c`` for the readings of the points the
paper leaves open.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

EQ1, MAX, FREQBIN, GREEDY, OPT = 0, 1, 2, 3, 4
GREEDY_FZ = 5   # 2D only: Greedy with fdot drift
VARIANTS = {"eq1": EQ1, "max": MAX, "freqbin": FREQBIN, "greedy": GREEDY, "opt": OPT,
            "greedy_fz": GREEDY_FZ}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrms_oracle.c")
_LIB = os.path.join(_HERE, "libhrms_oracle.so")

# Plain optimised C; no fast-math and no contraction, so every binary64 and
# binary32 operation is the IEEE one the source writes.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libhrms_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _configure(L):
    d, i64, i32, vp = C.c_double, C.c_int64, C.c_int, C.c_void_p
    L.oracle_num_levels.argtypes = [i32]
    L.oracle_stats.argtypes = [vp, i64, C.POINTER(d), C.POINTER(d)]
    L.oracle_snr_consts.argtypes = [i32, d, d, i32, vp, vp, vp, vp]
    L.oracle_sum_1d.argtypes = [vp, i64, i32, i32, i64, i32]
    L.oracle_sum_1d.restype = d
    L.oracle_sum_opt_paths.argtypes = [vp, i64, i32, i64, i32]
    L.oracle_sum_opt_paths.restype = d
    L.oracle_sum_2d.argtypes = [vp, i64, i32, i32, i32, i64, i32, i32]
    L.oracle_sum_2d.restype = d
    L.oracle_hrms_1d.argtypes = [vp, i64, i32, i32, vp, i64, vp, vp, i32, vp, vp, vp]
    L.oracle_hrms_2d.argtypes = [vp, i64, i64, i32, i32, i32, vp, vp, i64, vp, vp, i32,
                                 vp, vp, vp]
    L.oracle_scale_f32.argtypes = [vp, i64, d, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _configure(C.CDLL(_LIB))
    return _lib


class use_library:
    """Temporarily route every oracle call to another build of the oracle
    source (used by the tests that plant mistakes in a copy of it)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _configure(C.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def num_levels(hmax: int) -> int:
    n = lib().oracle_num_levels(int(hmax))
    if n < 1:
        raise ValueError(f"hmax must be a power of two <= 32, got {hmax}")
    return n


def levels(hmax: int):
    return [1 << k for k in range(num_levels(hmax))]


def stats(x):
    """Population mean and standard deviation (all bins)."""
    x = _f64(x).ravel()
    mu, sd = C.c_double(), C.c_double()
    if lib().oracle_stats(_ptr(x), x.size, C.byref(mu), C.byref(sd)) != 0:
        raise ValueError("oracle_stats: invalid input")
    return mu.value, sd.value


def snr_consts(variant: int, mu: float, sigma: float, hmax: int):
    """Null constants per level: (m32, q32, m64, q64)."""
    nl = num_levels(hmax)
    m32 = np.zeros(nl, np.float32)
    q32 = np.zeros(nl, np.float32)
    m64 = np.zeros(nl, np.float64)
    q64 = np.zeros(nl, np.float64)
    if lib().oracle_snr_consts(variant, mu, sigma, hmax, _ptr(m32), _ptr(q32), _ptr(m64),
                               _ptr(q64)) != 0:
        raise ValueError("oracle_snr_consts: invalid input")
    return m32, q32, m64, q64


def sum_1d(x, variant: int, H: int, n: int, f32: bool = False) -> float:
    """Unnormalised S_H(n) straight from the definition."""
    x = _f64(x)
    return lib().oracle_sum_1d(_ptr(x), x.size, variant, H, n, int(f32))


def sum_opt_paths(x, H: int, n: int, f32: bool = False) -> float:
    """Exhaustive-path S_H(n) by enumerating every offset path (H <= 24)."""
    x = _f64(x)
    return lib().oracle_sum_opt_paths(_ptr(x), x.size, H, n, int(f32))


def sum_2d(x2d, zmax: int, variant: int, H: int, m: int, z: int, f32: bool = False) -> float:
    x2d = _f64(x2d)
    return lib().oracle_sum_2d(_ptr(x2d), x2d.shape[1], zmax, variant, H, m, z, int(f32))


def hrms_1d(x, variant: int, hmax: int, idx=None, f32: bool = False, mu=None, sigma=None,
            want_snr: bool = True):
    """All levels of the outputs ``idx`` (default: every bin) of one spectrum.

    Returns ``(h, max_snr, best_h, consts)``; ``h`` has shape (levels, count)
    with NaN where a level does not exist. In FP32 mode the SNR uses the
    binary32 constants, in binary64 mode the binary64 ones. ``mu``/``sigma``
    default to the oracle's own statistics of ``x``.
    """
    x = _f64(x).ravel()
    N = x.size
    nl = num_levels(hmax)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        cnt = idx.size
    else:
        cnt = N
    consts = None
    mq = (None, None)
    if want_snr:
        if mu is None or sigma is None:
            mu, sigma = stats(x)
        consts = snr_consts(variant, mu, sigma, hmax)
        m32, q32, m64, q64 = consts
        mq = (m32.astype(np.float64), q32.astype(np.float64)) if f32 else (m64, q64)
    h = np.empty((nl, cnt), np.float64)
    ms = np.empty(cnt, np.float64)
    bh = np.empty(cnt, np.uint8)
    rc = lib().oracle_hrms_1d(_ptr(x), N, variant, hmax, _ptr(idx), cnt, _ptr(mq[0]),
                              _ptr(mq[1]), int(f32), _ptr(h), _ptr(ms), _ptr(bh))
    if rc != 0:
        raise ValueError("oracle_hrms_1d: invalid input")
    if not want_snr:
        ms = bh = None
    return h, ms, bh, consts


def hrms_2d(x2d, zmax: int, variant: int, hmax: int, fidx=None, zidx=None, f32: bool = False,
            mu=None, sigma=None, want_snr: bool = True):
    """All levels of plane outputs (m, z); whole plane when ``fidx`` is None.

    ``x2d`` has shape (2*zmax+1, nf). Whole-plane results are row-major over
    (z + zmax, m). For GREEDY_FZ the returned constants hold two sets of
    levels: the rows z != 0, then the row z = 0.
    """
    x2d = _f64(x2d)
    rows, nf = x2d.shape
    if rows != 2 * zmax + 1:
        raise ValueError("plane must have 2*zmax+1 rows")
    nl = num_levels(hmax)
    if fidx is not None:
        fidx = np.ascontiguousarray(fidx, dtype=np.int64)
        zidx = np.ascontiguousarray(zidx, dtype=np.int32)
        cnt = fidx.size
    else:
        cnt = rows * nf
    consts = None
    mq = (None, None)
    if want_snr:
        if mu is None or sigma is None:
            mu, sigma = stats(x2d)
        consts = snr_consts(variant, mu, sigma, hmax)
        m32, q32, m64, q64 = consts
        if variant == GREEDY_FZ:
            # the z = 0 row cannot drift in fdot: eq. (4)'s constants, as a
            # second set after the drifting rows' ones
            g32m, g32q, g64m, g64q = snr_consts(GREEDY, mu, sigma, hmax)
            m32, q32 = np.concatenate([m32, g32m]), np.concatenate([q32, g32q])
            m64, q64 = np.concatenate([m64, g64m]), np.concatenate([q64, g64q])
            consts = (m32, q32, m64, q64)
        mq = (m32.astype(np.float64), q32.astype(np.float64)) if f32 else (m64, q64)
    h = np.empty((nl, cnt), np.float64)
    ms = np.empty(cnt, np.float64)
    bh = np.empty(cnt, np.uint8)
    rc = lib().oracle_hrms_2d(_ptr(x2d), nf, nf, zmax, variant, hmax, _ptr(fidx), _ptr(zidx), cnt,
                              _ptr(mq[0]), _ptr(mq[1]), int(f32), _ptr(h), _ptr(ms), _ptr(bh))
    if rc != 0:
        raise ValueError("oracle_hrms_2d: invalid input")
    if not want_snr:
        ms = bh = None
    return h, ms, bh, consts


def candidates(max_snr, best_h, threshold: float):
    """The candidate list of one spectrum: every output whose maximum SNR over
    the levels reaches ``threshold`` (the thresholding that follows the
    harmonic sum in a search, Sec. 1), in increasing output order, as
    (bins, snr, best_h) arrays."""
    ms = np.asarray(max_snr)
    sel = np.nonzero(ms >= threshold)[0]
    return sel.astype(np.int64), ms[sel], np.asarray(best_h)[sel]


def peaks(max_snr, best_h, threshold: float):
    """The peak list of one spectrum: the candidates that are also local maxima
    of the maximum SNR along the spectrum -- max_snr[n] >= threshold,
    max_snr[n] > max_snr[n - 1] and max_snr[n] >= max_snr[n + 1], a missing
    neighbour at either end counting as lower (so a plateau keeps its lowest
    bin) -- in increasing output order, as (bins, snr, best_h) arrays. Written
    out one bin at a time."""
    ms = np.asarray(max_snr, dtype=np.float64)
    bh = np.asarray(best_h)
    out = []
    for n in range(ms.size):
        v = ms[n]
        lo = ms[n - 1] if n > 0 else -np.inf
        hi = ms[n + 1] if n + 1 < ms.size else -np.inf
        if v >= threshold and v > lo and v >= hi:
            out.append(n)
    sel = np.array(out, dtype=np.int64)
    return sel, ms[sel], bh[sel]


def scale_f32(x, mu: float):
    """binary32 product x * fl32(1/mu), before narrow rounding."""
    x = _f64(x).ravel()
    out = np.empty_like(x)
    if lib().oracle_scale_f32(_ptr(x), x.size, mu, _ptr(out)) != 0:
        raise ValueError("oracle_scale_f32: invalid input")
    return out
