"""Python binding of the C ABI in ``include/hrms.h`` (ctypes).

The functions carry the C names and only marshal arguments: every step of the
harmonic sum runs in the HIP kernels of ``libhrms.so``. PyTorch is used for
device memory and streams only. Loading fails loudly when the library has not
been built; there is no CPU fallback.

Paper: K. Adamek and W. Armour, arXiv:1812.02647 (eq. (1) in Sec. 1,
eq. (2)-(4) in Sec. 2).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhrms.so")

HRMS_EQ1, HRMS_MAX, HRMS_FREQBIN, HRMS_GREEDY, HRMS_OPT = 0, 1, 2, 3, 4
HRMS_GREEDY_FDOT = 5   # 2D only
HRMS_F32, HRMS_F16, HRMS_BF16 = 0, 1, 2
HRMS_OUT_H, HRMS_OUT_MAXSNR, HRMS_OUT_BESTH, HRMS_OUT_CAND, HRMS_OUT_PEAKS = 1, 2, 4, 8, 16
HRMS_OUT_ALL = 7
HRMS_STATS_COMPUTE, HRMS_STATS_PROVIDED = 0, 1
HRMS_OK, HRMS_E_INVAL, HRMS_E_UNSUPPORTED, HRMS_E_NODEVICE, HRMS_E_NOMEM, HRMS_E_HIP = (
    0, -1, -2, -3, -4, -5)
HRMS_MAX_LEVELS = 6
HRMS_MAX_BINS = 1 << 26

VARIANTS = {"eq1": HRMS_EQ1, "max": HRMS_MAX, "freqbin": HRMS_FREQBIN, "greedy": HRMS_GREEDY,
            "opt": HRMS_OPT, "greedy_fdot": HRMS_GREEDY_FDOT}
DTYPES = {"f32": HRMS_F32, "f16": HRMS_F16, "bf16": HRMS_BF16}

EXPORTED = ["hrms_create", "hrms_destroy", "hrms_layout_1d", "hrms_layout_2d", "hrms_run_1d",
            "hrms_run_1d_noalloc", "hrms_autotune_1d", "hrms_plan_1d", "hrms_run_2d", "hrms_quantize",
            "hrms_strerror", "hrms_last_error"]


class hrms_run1d_args(C.Structure):
    _fields_ = [
        ("n_spectra", C.c_int32),
        ("variant", C.c_int32),
        ("dtype", C.c_int32),
        ("hmax_all", C.c_int32),
        ("out_mask", C.c_uint32),
        ("stats_mode", C.c_int32),
        ("x", C.c_void_p),
        ("offsets", C.c_void_p),
        ("hmax", C.c_void_p),
        ("stats", C.c_void_p),
        ("snr_consts", C.c_void_p),
        ("h", C.c_void_p),
        ("max_snr", C.c_void_p),
        ("best_h", C.c_void_p),
        ("cand", C.c_void_p),
        ("cand_count", C.c_void_p),
        ("cand_capacity", C.c_uint32),
        ("cand_threshold", C.c_float),
    ]


class hrms_candidate(C.Structure):
    _fields_ = [("spectrum", C.c_int32), ("bin", C.c_int32), ("snr", C.c_float),
                ("best_h", C.c_int32)]


class hrms_run2d_args(C.Structure):
    _fields_ = [
        ("nf", C.c_int32),
        ("zmax", C.c_int32),
        ("hmax", C.c_int32),
        ("variant", C.c_int32),
        ("dtype", C.c_int32),
        ("out_mask", C.c_uint32),
        ("stats_mode", C.c_int32),
        ("reserved", C.c_int32),
        ("ld", C.c_int64),
        ("x", C.c_void_p),
        ("stats", C.c_void_p),
        ("snr_consts", C.c_void_p),
        ("h", C.c_void_p),
        ("max_snr", C.c_void_p),
        ("best_h", C.c_void_p),
    ]


class hrms_quantize_args(C.Structure):
    _fields_ = [
        ("n_spectra", C.c_int32),
        ("dtype", C.c_int32),
        ("stats_mode", C.c_int32),
        ("reserved", C.c_int32),
        ("x", C.c_void_p),
        ("offsets", C.c_void_p),
        ("stats", C.c_void_p),
        ("stats_out", C.c_void_p),
        ("y", C.c_void_p),
    ]


class HrmsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{strerror(status)} ({status}): {detail}")
        self.status = status


_lib = None


def lib():
    """The loaded ``libhrms.so``. Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() "
                "(or python -m paper_1812_02647_amd.build) first")
        # PyTorch ships its own copy of the HIP runtime. Loaded after this
        # library, it finds the runtime that this library pulled in and sees no
        # device; loading torch first makes both share torch's copy.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int
        L.hrms_create.argtypes = [C.POINTER(vp), i32, C.c_char_p]
        L.hrms_create.restype = i32
        L.hrms_destroy.argtypes = [vp]
        L.hrms_destroy.restype = i32
        L.hrms_layout_1d.argtypes = [C.POINTER(hrms_run1d_args), vp, C.POINTER(C.c_int64)]
        L.hrms_layout_1d.restype = i32
        L.hrms_layout_2d.argtypes = [C.POINTER(hrms_run2d_args), vp, C.POINTER(C.c_int64)]
        L.hrms_layout_2d.restype = i32
        L.hrms_run_1d.argtypes = [vp, C.POINTER(hrms_run1d_args), vp]
        L.hrms_run_1d.restype = i32
        L.hrms_run_1d_noalloc.argtypes = [vp, C.POINTER(hrms_run1d_args), vp]
        L.hrms_run_1d_noalloc.restype = i32
        L.hrms_autotune_1d.argtypes = [vp, C.POINTER(hrms_run1d_args), vp, i32,
                                       C.POINTER(C.c_int32)]
        L.hrms_autotune_1d.restype = i32
        L.hrms_plan_1d.argtypes = [vp, C.POINTER(hrms_run1d_args), C.POINTER(C.c_int32)]
        L.hrms_plan_1d.restype = i32
        L.hrms_run_2d.argtypes = [vp, C.POINTER(hrms_run2d_args), vp]
        L.hrms_run_2d.restype = i32
        L.hrms_quantize.argtypes = [vp, C.POINTER(hrms_quantize_args), vp]
        L.hrms_quantize.restype = i32
        L.hrms_strerror.argtypes = [i32]
        L.hrms_strerror.restype = C.c_char_p
        L.hrms_last_error.argtypes = [vp]
        L.hrms_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().hrms_strerror(status).decode()


def last_error(handle=None) -> str:
    return lib().hrms_last_error(handle).decode()


def _check(status: int, handle=None):
    if status != HRMS_OK:
        raise HrmsError(status, last_error(handle))


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------

def hrms_create(device: int = 0, tune_cache_path: str | None = None):
    h = C.c_void_p()
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().hrms_create(C.byref(h), device, path))
    return h


def hrms_destroy(handle) -> None:
    _check(lib().hrms_destroy(handle))


def hrms_layout_1d(args: hrms_run1d_args):
    n = args.n_spectra
    offs = np.empty((max(n, 0), HRMS_MAX_LEVELS), np.int64)
    total = C.c_int64()
    _check(lib().hrms_layout_1d(C.byref(args), offs.ctypes.data_as(C.c_void_p), C.byref(total)))
    return offs, total.value


def hrms_layout_2d(args: hrms_run2d_args):
    offs = np.empty(HRMS_MAX_LEVELS, np.int64)
    total = C.c_int64()
    _check(lib().hrms_layout_2d(C.byref(args), offs.ctypes.data_as(C.c_void_p), C.byref(total)))
    return offs, total.value


def hrms_run_1d(handle, args: hrms_run1d_args, stream=None) -> None:
    _check(lib().hrms_run_1d(handle, C.byref(args), _stream_ptr(stream)), handle)


def hrms_run_1d_noalloc(handle, args: hrms_run1d_args, stream=None) -> None:
    _check(lib().hrms_run_1d_noalloc(handle, C.byref(args), _stream_ptr(stream)), handle)


def hrms_autotune_1d(handle, args: hrms_run1d_args, stream=None, reps: int = 3):
    """Times every compiled launch shape on this batch and keeps the fastest;
    returns (wg, r, chunk, top)."""
    chosen = (C.c_int32 * 4)()
    _check(lib().hrms_autotune_1d(handle, C.byref(args), _stream_ptr(stream), reps, chosen),
           handle)
    return tuple(chosen)


def hrms_plan_1d(handle, args: hrms_run1d_args):
    """The launches hrms_run_1d would make for this batch:
    ((wg, r, chunk, top), number of harmonic-sum launches)."""
    info = (C.c_int32 * 5)()
    _check(lib().hrms_plan_1d(handle, C.byref(args), info), handle)
    return tuple(info[:4]), int(info[4])


def hrms_run_2d(handle, args: hrms_run2d_args, stream=None) -> None:
    _check(lib().hrms_run_2d(handle, C.byref(args), _stream_ptr(stream)), handle)


def hrms_quantize(handle, args: hrms_quantize_args, stream=None) -> None:
    _check(lib().hrms_quantize(handle, C.byref(args), _stream_ptr(stream)), handle)


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:  # pragma: no cover - no torch / no device
            return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Tensor-level convenience (argument marshalling and output allocation)
# ---------------------------------------------------------------------------

_TORCH_DT = None


def _torch_dtype_code(t):
    import torch
    m = {torch.float32: HRMS_F32, torch.float16: HRMS_F16, torch.bfloat16: HRMS_BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported input dtype {t.dtype}")
    return m[t.dtype]


def _check_input(x, offsets) -> None:
    """The library builds buffer resources from the offsets and cannot see
    the tensor behind a pointer: x must be a contiguous device tensor holding
    every bin the offsets name."""
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("x must be a torch tensor")
    if x.device.type != "cuda":
        raise ValueError(f"x must be on a HIP device, not {x.device}")
    _check_input_layout(x, offsets)


def _check_input_layout(x, offsets) -> None:
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    if offsets.ndim != 1 or offsets.size < 2:
        raise ValueError("offsets must hold n_spectra + 1 >= 2 values")
    if x.numel() < int(offsets[-1]):
        raise ValueError(f"x holds {x.numel()} bins, the offsets name {int(offsets[-1])}")


def _check_stats(stats, shape, device) -> None:
    import torch
    if not isinstance(stats, torch.Tensor) or stats.dtype != torch.float64:
        raise TypeError("stats must be a float64 torch tensor")
    if tuple(stats.shape) != tuple(shape):
        raise ValueError(f"stats must have shape {tuple(shape)}, not {tuple(stats.shape)}")
    if stats.device != device:
        raise ValueError(f"stats must be on {device}, not {stats.device}")
    if not stats.is_contiguous():
        raise ValueError("stats must be contiguous")


class Batch1D:
    """Device buffers of one 1D batch call. ``offsets`` and ``hmax`` stay on the
    host (numpy); ``x`` and every output are torch tensors on the device."""

    def __init__(self, x, offsets, variant, hmax, out_mask=HRMS_OUT_ALL, stats=None,
                 want_consts=True, cand_capacity=0, cand_threshold=6.0):
        import torch
        self.x = x
        self.offsets = np.ascontiguousarray(offsets, np.int64)
        n = self.offsets.size - 1
        _check_input(x, self.offsets)
        if stats is not None:
            _check_stats(stats, (n, 2), x.device)
        if np.isscalar(hmax):
            self.hmax_arr = None
            self.hmax_all = int(hmax)
        else:
            self.hmax_arr = np.ascontiguousarray(hmax, np.uint8)
            self.hmax_all = 0
        self.args = hrms_run1d_args()
        a = self.args
        a.n_spectra = n
        a.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        a.dtype = _torch_dtype_code(x)
        a.hmax_all = self.hmax_all
        a.out_mask = out_mask
        a.stats_mode = HRMS_STATS_PROVIDED if stats is not None else HRMS_STATS_COMPUTE
        a.x = x.data_ptr()
        a.offsets = self.offsets.ctypes.data
        a.hmax = self.hmax_arr.ctypes.data if self.hmax_arr is not None else None
        self.plane_offsets, self.h_total = hrms_layout_1d(a)
        dev = x.device
        total = int(self.offsets[-1])
        self.stats = stats if stats is not None else torch.zeros(
            (n, 2), dtype=torch.float64, device=dev)
        self.consts = torch.zeros((n, HRMS_MAX_LEVELS, 2), dtype=torch.float32,
                                  device=dev) if want_consts else None
        self.h = torch.empty(max(self.h_total, 1), dtype=torch.float32, device=dev) \
            if out_mask & HRMS_OUT_H else None
        self.max_snr = torch.empty(total, dtype=torch.float32, device=dev) \
            if out_mask & HRMS_OUT_MAXSNR else None
        self.best_h = torch.empty(total, dtype=torch.uint8, device=dev) \
            if out_mask & HRMS_OUT_BESTH else None
        # candidate list: records of 4 int32 words (spectrum, bin, snr bits, best H)
        listing = (out_mask & (HRMS_OUT_CAND | HRMS_OUT_PEAKS)) != 0
        self.cand = torch.zeros((max(cand_capacity, 1), 4), dtype=torch.int32, device=dev) \
            if listing else None
        self.cand_count = torch.zeros(1, dtype=torch.int32, device=dev) if listing else None
        a.cand = self.cand.data_ptr() if self.cand is not None else None
        a.cand_count = self.cand_count.data_ptr() if self.cand_count is not None else None
        a.cand_capacity = cand_capacity if listing else 0
        a.cand_threshold = cand_threshold
        a.stats = self.stats.data_ptr()
        a.snr_consts = self.consts.data_ptr() if self.consts is not None else None
        a.h = self.h.data_ptr() if self.h is not None else None
        a.max_snr = self.max_snr.data_ptr() if self.max_snr is not None else None
        a.best_h = self.best_h.data_ptr() if self.best_h is not None else None

    def run(self, handle, stream=None):
        hrms_run_1d(handle, self.args, stream)
        return self

    def run_noalloc(self, handle, stream=None):
        hrms_run_1d_noalloc(handle, self.args, stream)
        return self

    def candidates(self):
        """(count, records): records as a numpy structured array of the first
        min(count, capacity) candidates, in the order the kernels wrote them."""
        n = int(self.cand_count.cpu()[0])
        raw = self.cand[:min(n, self.args.cand_capacity)].cpu().numpy()
        rec = np.empty(raw.shape[0], dtype=[("spectrum", np.int32), ("bin", np.int32),
                                             ("snr", np.float32), ("best_h", np.int32)])
        rec["spectrum"], rec["bin"], rec["best_h"] = raw[:, 0], raw[:, 1], raw[:, 3]
        rec["snr"] = raw[:, 2].view(np.float32)
        return n, rec

    def level(self, s: int, l: int):
        """Level l (H = 2^l) plane of spectrum s, as a view of ``h``."""
        o = int(self.plane_offsets[s, l])
        if o < 0:
            return None
        n = int(self.offsets[s + 1] - self.offsets[s])
        ln = n if self.args.variant == HRMS_EQ1 else n >> l
        return self.h[o:o + ln]
