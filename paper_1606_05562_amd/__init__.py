"""MI355X (gfx950) implementation of the orthogonal 16-point approximate DCT
(da Silveira et al., "An Orthogonal 16-point Approximate DCT for Image and
Video Compression").

This module is a thin ctypes binding of the C ABI declared in
include/adct16.h: it marshals arguments (device pointers of torch tensors,
the current HIP stream) and raises on error status.  Every step of the
transform runs in the HIP library libadct16.so.  The library is loaded on
first use, so that the build step (paper_1606_05562_amd.build) can run in a
tree where it does not exist yet; any call made while it is missing raises
ImportError.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadct16.so")

# adct16_status
OK, E_NULL, E_SHAPE, E_DTYPE, E_MODE, E_ALIGN, E_NOMEM, E_DEVICE, E_LAUNCH, E_STATE = range(10)
# adct16_dtype
U8, I16, I32, F32, BF16, F16 = 1, 2, 3, 4, 5, 6
# adct16_qmode
Q_NONE, Q_ZONAL, Q_ZIGZAG, Q_UNIFORM, Q_DEADZONE = 0, 1, 2, 3, 4
# adct16_backend
BACKEND_AUTO, BACKEND_VALU, BACKEND_MFMA = 0, 1, 2
FLAG_AUTOTUNE = 1
FLAG_EXPLICIT_COEF = 2
FLAG_MFMA_INT8 = 4
FLAG_DEADZONE_INTER = 8
FLAG_RESIDUAL_RANGE = 16
# adct16_matrix
MATRIX_APPROX, MATRIX_T, MATRIX_WHT, MATRIX_DCT = 0, 1, 2, 3

_TORCH_DTYPE_CODES = {"torch.uint8": U8, "torch.int16": I16, "torch.int32": I32, "torch.float32": F32}

EXPORTED = [
    "adct16_plan_create", "adct16_plan_destroy", "adct16_plan_num_blocks", "adct16_plan_info",
    "adct16_plan_time_fused", "adct16_plan_fused_times",
    "adct16_forward", "adct16_quantise", "adct16_inverse", "adct16_measure", "adct16_rate",
    "adct16_dct_compress_and_measure", "adct16_ssim",
    "adct16_compress_and_measure", "adct16_compress_and_measure_static", "adct16_dct_forward", "adct16_forward_1d", "adct16_inverse_1d",
    "adct16_graph_create", "adct16_graph_launch", "adct16_graph_destroy",
    "adct16_transform_matrix", "adct16_transform_measures",
    "adct16_status_string", "adct16_last_error_string",
]


class Adct16Error(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"adct16 status {status}: {message}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n_images", ctypes.c_int32),
        ("height", ctypes.POINTER(ctypes.c_int32)),
        ("width", ctypes.POINTER(ctypes.c_int32)),
        ("pitch", ctypes.POINTER(ctypes.c_int32)),
        ("offset", ctypes.POINTER(ctypes.c_int64)),
        ("in_dtype", ctypes.c_int32),
        ("coef_dtype", ctypes.c_int32),
        ("qcoef_dtype", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
        ("qmode", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("backend", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("matrix", ctypes.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_1606_05562_amd.build.build() "
                          "(hipcc, gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "adct16_plan_create": [ctypes.POINTER(_Desc), ctypes.POINTER(vp)],
        "adct16_plan_destroy": [vp],
        "adct16_plan_num_blocks": [vp, ctypes.POINTER(i64)],
        "adct16_plan_info": [vp, ctypes.c_char_p, i32],
        "adct16_plan_time_fused": [vp, i32],
        "adct16_plan_fused_times": [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)],
        "adct16_forward": [vp, vp, vp, vp],
        "adct16_quantise": [vp, vp, vp, vp],
        "adct16_inverse": [vp, vp, vp, vp],
        "adct16_measure": [vp, vp, vp, vp, vp, vp],
        "adct16_rate": [vp, vp, vp, vp],
        "adct16_dct_compress_and_measure": [vp, vp, vp, vp, vp, vp],
        "adct16_ssim": [vp, vp, vp, vp, vp],
        "adct16_compress_and_measure": [vp, vp, vp, vp, vp, vp, vp],
        "adct16_compress_and_measure_static": [vp, vp, vp, vp, vp, vp, vp],
        "adct16_dct_forward": [vp, vp, vp, i32, vp],
        "adct16_forward_1d": [vp, vp, i64, vp],
        "adct16_inverse_1d": [vp, vp, i64, vp],
        "adct16_graph_create": [vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)],
        "adct16_graph_launch": [vp, vp],
        "adct16_graph_destroy": [vp],
        "adct16_transform_matrix": [i32, ctypes.POINTER(ctypes.c_double)],
        "adct16_transform_measures": [ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.adct16_status_string.argtypes = [ctypes.c_int]
    lib.adct16_status_string.restype = ctypes.c_char_p
    lib.adct16_last_error_string.argtypes = []
    lib.adct16_last_error_string.restype = ctypes.c_char_p
    return lib


_LIB = None


def lib():
    """The loaded libadct16.so (loaded on the first call; raises ImportError
    if it has not been built)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def _check(st: int):
    if st != OK:
        raise Adct16Error(st, f"{lib().adct16_status_string(st).decode()}: {lib().adct16_last_error_string().decode()}")


def _ptr(t) -> int | None:
    """Device address of a tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """A batch description (image sizes and layout, dtypes, quantiser) bound
    to the current device.  See include/adct16.h for every field."""

    def __init__(self, heights, widths, pitches, offsets, in_dtype=U8, coef_dtype=I32,
                 qcoef_dtype=None, out_dtype=None, qmode=Q_NONE, r=16, q=1,
                 backend=BACKEND_AUTO, flags=0, matrix=MATRIX_APPROX):
        n = len(heights)
        if not (len(widths) == len(pitches) == len(offsets) == n):
            raise ValueError("heights, widths, pitches and offsets must have equal lengths")
        self._h = (ctypes.c_int32 * max(n, 1))(*heights)
        self._w = (ctypes.c_int32 * max(n, 1))(*widths)
        self._p = (ctypes.c_int32 * max(n, 1))(*pitches)
        self._o = (ctypes.c_int64 * max(n, 1))(*offsets)
        if qcoef_dtype is None:
            qcoef_dtype = I16 if qmode in (Q_UNIFORM, Q_DEADZONE) else (coef_dtype if coef_dtype in (I32, I16) else I32)
        if out_dtype is None:
            out_dtype = in_dtype
        d = _Desc(n, self._h, self._w, self._p, self._o, in_dtype, coef_dtype, qcoef_dtype, out_dtype,
                  qmode, r, q, backend, flags, matrix)
        h = ctypes.c_void_p()
        _check(lib().adct16_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._plan = h
        self.n_images = n
        self.in_dtype, self.coef_dtype, self.qcoef_dtype, self.out_dtype = in_dtype, coef_dtype, qcoef_dtype, out_dtype
        self.qmode, self.r, self.q = qmode, r, q

    def close(self):
        if getattr(self, "_plan", None):
            lib().adct16_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_blocks(self) -> int:
        n = ctypes.c_int64()
        _check(lib().adct16_plan_num_blocks(self._plan, ctypes.byref(n)))
        return n.value

    def info(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(lib().adct16_plan_info(self._plan, buf, len(buf)))
        return buf.value.decode()

    def time_fused(self, n_calls: int):
        """Record the persistent kernel's duration on the next n_calls fused calls."""
        _check(lib().adct16_plan_time_fused(self._plan, n_calls))

    def fused_times(self, cap: int = 65536) -> list[float]:
        """Kernel durations (ms) of the calls recorded since time_fused (or
        the previous read); waits for them."""
        ms = (ctypes.c_float * max(cap, 1))()
        n = ctypes.c_int32()
        _check(lib().adct16_plan_fused_times(self._plan, ms, cap, ctypes.byref(n)))
        return list(ms[:min(n.value, cap)])

    def forward(self, inp, coef, stream=None):
        _check(lib().adct16_forward(self._plan, _ptr(inp), _ptr(coef), _stream(stream)))

    def quantise(self, coef, qcoef, stream=None):
        _check(lib().adct16_quantise(self._plan, _ptr(coef), _ptr(qcoef), _stream(stream)))

    def inverse(self, qcoef, out, stream=None):
        _check(lib().adct16_inverse(self._plan, _ptr(qcoef), _ptr(out), _stream(stream)))

    def measure(self, a, b, sse, psnr=None, stream=None):
        _check(lib().adct16_measure(self._plan, _ptr(a), _ptr(b), _ptr(sse), _ptr(psnr), _stream(stream)))

    def dct_compress_and_measure(self, inp, out=None, sse=None, psnr=None, stream=None):
        """The same retention with the exact DCT-II in float64 (comparison)."""
        _check(lib().adct16_dct_compress_and_measure(self._plan, _ptr(inp), _ptr(out), _ptr(sse), _ptr(psnr),
                                                    _stream(stream)))

    def ssim(self, a, b, out, stream=None):
        """Per-image mean SSIM (float64) of b against a."""
        _check(lib().adct16_ssim(self._plan, _ptr(a), _ptr(b), _ptr(out), _stream(stream)))

    def rate(self, qcoef, bits, stream=None):
        """Per-image signed Exp-Golomb code length (bits, int64) of the levels."""
        _check(lib().adct16_rate(self._plan, _ptr(qcoef), _ptr(bits), _stream(stream)))

    def compress_and_measure(self, inp, out=None, qcoef=None, sse=None, psnr=None, stream=None):
        _check(lib().adct16_compress_and_measure(self._plan, _ptr(inp), _ptr(out), _ptr(qcoef), _ptr(sse),
                                                _ptr(psnr), _stream(stream)))

    def compress_and_measure_static(self, inp, out=None, qcoef=None, sse=None, psnr=None, stream=None):
        """compress_and_measure with the library's fixed device scratch array
        (no allocation); calls that overlap on one GPU race."""
        _check(lib().adct16_compress_and_measure_static(self._plan, _ptr(inp), _ptr(out), _ptr(qcoef), _ptr(sse),
                                                       _ptr(psnr), _stream(stream)))

    def dct_forward(self, inp, y, precision=F16, stream=None):
        _check(lib().adct16_dct_forward(self._plan, _ptr(inp), _ptr(y), precision, _stream(stream)))

    def graph(self, inp, out=None, qcoef=None, sse=None, psnr=None):
        return Graph(self, inp, out, qcoef, sse, psnr)


class Graph:
    """adct16_compress_and_measure captured with fixed buffers in a HIP graph."""

    def __init__(self, plan: Plan, inp, out=None, qcoef=None, sse=None, psnr=None):
        g = ctypes.c_void_p()
        _check(lib().adct16_graph_create(plan._plan, _ptr(inp), _ptr(out), _ptr(qcoef), _ptr(sse), _ptr(psnr),
                                        ctypes.byref(g)))
        self._g = g
        self._keep = (plan, inp, out, qcoef, sse, psnr)

    def launch(self, stream=None):
        _check(lib().adct16_graph_launch(self._g, _stream(stream)))

    def close(self):
        if getattr(self, "_g", None):
            lib().adct16_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_1d(x, y, stream=None):
    """y = T x for each row of an (n, 16) int32 device tensor."""
    _check(lib().adct16_forward_1d(_ptr(x), _ptr(y), x.shape[0], _stream(stream)))


def inverse_1d(x, y, stream=None):
    """y = T^T x for each row of an (n, 16) int32 device tensor."""
    _check(lib().adct16_inverse_1d(_ptr(x), _ptr(y), x.shape[0], _stream(stream)))


def transform_matrix(which: int = MATRIX_APPROX):
    """The 16x16 matrix ``which`` (MATRIX_APPROX, MATRIX_T, MATRIX_WHT,
    MATRIX_DCT) as a float64 numpy array."""
    import numpy as np
    m = np.empty((16, 16), dtype=np.float64)
    _check(lib().adct16_transform_matrix(which, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return m


def transform_measures(ct, rho: float = 0.95) -> dict:
    """Table 2 measures of the 16x16 transform ``ct`` against the DCT-II:
    d2, epsilon (total error energy), mse, cg (coding gain, dB), eta
    (transform efficiency, %)."""
    import numpy as np
    a = np.ascontiguousarray(ct, dtype=np.float64)
    if a.shape != (16, 16):
        raise ValueError("ct must be 16x16")
    out = np.empty(5, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().adct16_transform_measures(a.ctypes.data_as(dp), float(rho), out.ctypes.data_as(dp)))
    return dict(zip(("d2", "epsilon", "mse", "cg", "eta"), out.tolist()))


def status_string(st: int) -> str:
    return lib().adct16_status_string(st).decode()
