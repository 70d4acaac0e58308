"""Width-5 separable image convolution on AMD Instinct MI355X (gfx950).

A thin ctypes binding over ``libconvsep5.so`` (C ABI in ``include/conv_sep5.h``).
The functions carry the C names and only marshal arguments: every step of the
convolution runs in the library's HIP kernels.  torch tensors supply device
memory and streams.  If the library is not built, every call raises.

Image tensors are [planes, rows, cols] (float32, float16 or bfloat16) on the
GPU with unit column stride; row and plane strides become the descriptor's
pitch and plane_stride.  Taps are 5 FP32 numbers; k[0] weights the neighbour at
offset -2 (correlation form of Eq. 1, arXiv 1711.09791).
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libconvsep5.so")
LOADGEN_PATH = os.path.join(_PKG, "libconvsep5_loadgen.so")

CONV_OK, CONV_EINVAL, CONV_EALIAS, CONV_ENOMEM = 0, -1, -2, -3
CONV_EHIP, CONV_EAGAIN, CONV_ENOTFOUND = -4, -5, -6
CONV_F32, CONV_F16, CONV_BF16 = 0, 1, 2
CONV_1PASS_FUSED, CONV_1PASS_DIRECT25 = 0, 1
# bytes of the static device workspace of conv_sep5_2pass_noalloc (per GPU)
CONV_NOALLOC_SCRATCH_BYTES = 128 << 20
KIND_IMAGE, KIND_BATCH, KIND_DIRECT = 0, 1, 2

_STATUS_NAMES = {0: "CONV_OK", -1: "CONV_EINVAL", -2: "CONV_EALIAS", -3: "CONV_ENOMEM",
                 -4: "CONV_EHIP", -5: "CONV_EAGAIN", -6: "CONV_ENOTFOUND"}


class conv_image(ctypes.Structure):
    _fields_ = [("planes", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("pitch", ctypes.c_int64), ("plane_stride", ctypes.c_int64)]


class conv_tile_cfg(ctypes.Structure):
    _fields_ = [("rows_per_tile", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32),
                ("persist_wgs_per_cu", ctypes.c_int32), ("xcd_slabs", ctypes.c_int32),
                ("pack_tail", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class conv_serve_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_batch_bytes", ctypes.c_uint64),
                ("producer_wait", ctypes.c_int32), ("queue_only", ctypes.c_int32),
                ("launch_depth", ctypes.c_int32)]


class conv_req_times(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("launch_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64),
                ("batch_size", ctypes.c_int32), ("stream", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class conv_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("max_bytes_in_flight", ctypes.c_uint64), ("max_slots_in_flight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_streams_busy", ctypes.c_int32),
                ("direct_launches", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ConvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

EXPORTS = (
    "conv_sep5_2pass", "conv_sep5_2pass_ex", "conv_sep5_2pass_noalloc", "conv_sep5_1pass",
    "conv_image_copy",
    "conv_sep5_batch",
    "conv_batch_plan_create", "conv_batch_plan_launch", "conv_batch_plan_destroy",
    "conv_sepn_1pass", "conv_sepn_2pass", "conv_2d_direct", "conv_pyr_down",
    "conv_get_tile_cfg", "conv_set_tile_cfg", "conv_get_tile_cfg_for", "conv_tune",
    "conv_tune_save", "conv_tune_load",
    "conv_serve_create", "conv_serve_submit", "conv_serve_poll", "conv_serve_drain",
    "conv_serve_destroy", "conv_serve_get_stats", "conv_last_error", "conv_version",
)


def lib():
    """The loaded libconvsep5.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libconvsep5.so is not built ({LIB_PATH}); run `python -m "
            "paper_1711_09791_amd.build` or __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    fp = ctypes.POINTER(ctypes.c_float)
    imgp = ctypes.POINTER(conv_image)
    cfgp = ctypes.POINTER(conv_tile_cfg)
    sig = {
        "conv_sep5_2pass": [vp, vp, vp, fp, imgp, vp],
        "conv_sep5_2pass_ex": [vp, vp, vp, fp, imgp, i32, vp],
        "conv_sep5_2pass_noalloc": [vp, vp, fp, imgp, i32, vp],
        "conv_sep5_1pass": [vp, vp, fp, imgp, ctypes.c_int, vp],
        "conv_image_copy": [vp, vp, imgp, vp],
        "conv_sep5_batch": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), fp, imgp, ctypes.c_int, vp],
        "conv_batch_plan_create": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), fp, imgp,
                                   ctypes.c_int, ctypes.POINTER(vp)],
        "conv_sepn_1pass": [vp, vp, fp, i32, imgp, ctypes.c_int, vp],
        "conv_sepn_2pass": [vp, vp, vp, fp, i32, imgp, vp],
        "conv_2d_direct": [vp, vp, fp, i32, imgp, vp],
        "conv_pyr_down": [vp, imgp, vp, imgp, fp, vp],
        "conv_batch_plan_launch": [vp, vp],
        "conv_batch_plan_destroy": [vp],
        "conv_get_tile_cfg": [i32, i32, cfgp],
        "conv_set_tile_cfg": [i32, i32, cfgp],
        "conv_get_tile_cfg_for": [i32, i32, u64, cfgp, ctypes.POINTER(i32)],
        "conv_tune_save": [ctypes.c_char_p],
        "conv_tune_load": [ctypes.c_char_p],
        "conv_tune": [i32, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), fp, imgp, i32, vp, cfgp,
                      fp],
        "conv_serve_create": [ctypes.POINTER(conv_serve_cfg), ctypes.POINTER(vp)],
        "conv_serve_submit": [vp, vp, vp, fp, imgp, vp, ctypes.POINTER(u64)],
        "conv_serve_poll": [vp, u64, ctypes.POINTER(conv_req_times)],
        "conv_serve_drain": [vp],
        "conv_serve_destroy": [vp],
        "conv_serve_get_stats": [vp, ctypes.POINTER(conv_serve_stats)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.conv_last_error.argtypes = []
    L.conv_last_error.restype = ctypes.c_char_p
    L.conv_version.argtypes = []
    L.conv_version.restype = ctypes.c_char_p
    _lib = L
    return L


_loadgen = None

LOADGEN_EXPORTS = ("conv_loadgen_serve", "conv_loadgen_direct", "conv_loadgen_call_latency")


def loadgen_lib():
    """libconvsep5_loadgen.so (open-loop request generator for benchmarks)."""
    global _loadgen
    if _loadgen is not None:
        return _loadgen
    lib()
    if not os.path.exists(LOADGEN_PATH):
        raise RuntimeError(f"{LOADGEN_PATH} is not built")
    G = ctypes.CDLL(LOADGEN_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    G.conv_loadgen_serve.argtypes = [vp, i32, dp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(ctypes.c_float), ctypes.POINTER(conv_image),
                                     vp, u64p, dp]
    G.conv_loadgen_serve.restype = ctypes.c_int
    G.conv_loadgen_direct.argtypes = [i32, dp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(ctypes.c_float), ctypes.POINTER(conv_image),
                                      i32, u64p, u64p, dp]
    G.conv_loadgen_direct.restype = ctypes.c_int
    G.conv_loadgen_call_latency.argtypes = [i32, i32, vp, vp, vp, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(conv_image), vp, dp, dp]
    G.conv_loadgen_call_latency.restype = ctypes.c_int
    _loadgen = G
    return G


def conv_last_error() -> str:
    return lib().conv_last_error().decode()


def _check(st: int) -> int:
    if st != CONV_OK:
        raise ConvError(st, conv_last_error())
    return st


# ---- argument marshalling ------------------------------------------------------------

def _dtype_code(t) -> int:
    import torch

    m = {torch.float32: CONV_F32, torch.float16: CONV_F16, torch.bfloat16: CONV_BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _no_broadcast(shape, strides) -> None:
    """A zero stride in a dimension of size > 1 (an expanded or broadcast view)
    repeats memory; the descriptor reads 0 as the dense default and would
    cover bytes the tensor does not own."""
    for n, s in zip(shape, strides):
        if n > 1 and s == 0:
            raise ValueError(f"zero stride in a dimension of size {n} (broadcast or expanded "
                             "view); pass a contiguous tensor")


def image_of(t) -> conv_image:
    """conv_image describing a [planes, rows, cols] (or [rows, cols]) tensor."""
    if t.dim() in (2, 3) and t.numel() == 0:
        shape = (1, *t.shape) if t.dim() == 2 else tuple(t.shape)
        return conv_image(*(int(v) for v in shape), _dtype_code(t), 0, 0)
    if t.dim() == 2:
        P, (R, C) = 1, t.shape
        sp, sr, sc = R * t.stride(0), t.stride(0), t.stride(1)
    elif t.dim() == 3:
        P, R, C = t.shape
        sp, sr, sc = t.stride()
    else:
        raise ValueError("image tensors are [planes, rows, cols] or [rows, cols]")
    if C > 1 and sc != 1:
        raise ValueError("columns must be contiguous (unit stride); use image_hwc for "
                         "pixel-interleaved [rows, cols, planes] tensors")
    _no_broadcast((P, R, C), (sp, sr, sc))
    if P > 1 and C > 1 and sp == 1:
        raise ValueError("plane stride 1 with contiguous columns makes planes overlap")
    if P > 1 and R == 1 and C == 1:
        # one pixel per plane: any plane stride is the dense planar layout
        return conv_image(int(P), 1, 1, _dtype_code(t), 1, 0)
    return conv_image(int(P), int(R), int(C), _dtype_code(t), int(sr) if R > 1 else int(C),
                      int(sp) if P > 1 else 0)


def image_hwc(t) -> conv_image:
    """conv_image of a pixel-interleaved [rows, cols, planes] tensor (packed
    HWC: planes 2..4 contiguous per pixel, pixels contiguous in a row); the
    descriptor's plane_stride is 1."""
    if t.dim() != 3:
        raise ValueError("HWC image tensors are [rows, cols, planes]")
    R, C, P = (int(v) for v in t.shape)
    if t.numel() == 0:
        return conv_image(P, R, C, _dtype_code(t), 0, 1)
    sr, sc, sp = t.stride()
    _no_broadcast((R, C, P), (sr, sc, sp))
    if (P > 1 and sp != 1) or (C > 1 and sc != P):
        raise ValueError("HWC tensors need contiguous pixels (strides [pitch, planes, 1])")
    return conv_image(P, R, C, _dtype_code(t), int(sr) if R > 1 else C * P, 1)


def _same_layout(a, b, what: str = "output") -> None:
    """The C ABI describes input and output with ONE descriptor: a tensor pair
    must agree in shape, dtype, device and strides (raw pointers are the
    caller's responsibility)."""
    if isinstance(a, int) or isinstance(b, int) or a is None or b is None:
        return
    if tuple(a.shape) != tuple(b.shape) or a.dtype != b.dtype or a.device != b.device:
        raise ValueError(f"{what} must match the input's shape, dtype and device "
                         f"({tuple(b.shape)} {b.dtype} vs {tuple(a.shape)} {a.dtype})")
    if a.numel() and tuple(a.stride()) != tuple(b.stride()):
        raise ValueError(f"{what} strides {tuple(b.stride())} differ from the input's "
                         f"{tuple(a.stride())}; both share one layout descriptor")


def _taps(k) -> ctypes.Array:
    vals = [float(v) for v in (k.tolist() if hasattr(k, "tolist") else k)]
    if len(vals) != 5:
        raise ValueError("k must hold 5 taps")
    return (ctypes.c_float * 5)(*vals)


def _taps_n(k) -> tuple[ctypes.Array, int]:
    """Any number of FP32 taps (the library checks the width)."""
    vals = [float(v) for v in (k.reshape(-1).tolist() if hasattr(k, "reshape") else k)]
    return (ctypes.c_float * max(len(vals), 1))(*vals), len(vals)


def _kernel_nn(K) -> tuple[ctypes.Array, int]:
    """A square n x n kernel (nested sequence, array or tensor) -> row-major FP32."""
    rows = K.tolist() if hasattr(K, "tolist") else [list(r) for r in K]
    n = len(rows)
    if any(len(r) != n for r in rows):
        raise ValueError("K must be a square n x n kernel")
    vals = [float(v) for r in rows for v in r]
    return (ctypes.c_float * max(len(vals), 1))(*vals), n


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(x):
    if x is None:
        return ctypes.c_void_p(0)
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    return ctypes.c_void_p(x.data_ptr())


# ---- entry points ----------------------------------------------------------------------

def _check_workspace(d_tmp, img: conv_image, esz: int) -> None:
    """A workspace tensor is raw device memory for planes*rows*cols values of
    the intermediate's type (esz bytes each): the library writes that many
    bytes from its start, so it must be contiguous and at least that large."""
    if d_tmp is None or isinstance(d_tmp, int):
        return
    need = int(img.planes) * int(img.rows) * int(img.cols) * esz
    have = d_tmp.numel() * d_tmp.element_size()
    if have < need:
        raise ValueError(f"workspace holds {have} bytes, the intermediate needs {need}")
    if not d_tmp.is_contiguous():
        raise ValueError("workspace must be contiguous")


def conv_sep5_2pass(d_in, d_out, k, d_tmp=None, img: conv_image | None = None, stream=None):
    """Two-pass form: row kernel into the FP32 workspace, then column kernel."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    _check_workspace(d_tmp, img, 4)
    return _check(lib().conv_sep5_2pass(_ptr(d_in), _ptr(d_out), _ptr(d_tmp), _taps(k),
                                        ctypes.byref(img), _stream(stream)))


def conv_sep5_2pass_ex(d_in, d_out, k, tmp_dtype: int, d_tmp=None,
                       img: conv_image | None = None, stream=None):
    """Two-pass form with the intermediate stored as tmp_dtype (CONV_F32,
    CONV_F16 or CONV_BF16); d_tmp holds planes*rows*cols values of it."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    if int(tmp_dtype) in (CONV_F32, CONV_F16, CONV_BF16):
        _check_workspace(d_tmp, img, 4 if int(tmp_dtype) == CONV_F32 else 2)
    return _check(lib().conv_sep5_2pass_ex(_ptr(d_in), _ptr(d_out), _ptr(d_tmp), _taps(k),
                                           ctypes.byref(img), int(tmp_dtype), _stream(stream)))


def conv_sep5_2pass_noalloc(d_in, d_out, k, tmp_dtype: int = CONV_F32,
                            img: conv_image | None = None, stream=None):
    """Two-pass form with the intermediate in the library's static device
    workspace (CONV_NOALLOC_SCRATCH_BYTES per GPU): allocates nothing.  Calls
    that can overlap on one GPU race on that workspace."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    return _check(lib().conv_sep5_2pass_noalloc(_ptr(d_in), _ptr(d_out), _taps(k), ctypes.byref(img),
                                                int(tmp_dtype), _stream(stream)))


def conv_sep5_1pass(d_in, d_out, k, mode: int = CONV_1PASS_FUSED,
                    img: conv_image | None = None, stream=None):
    """Single-pass form (fused row+column, or the direct 25-tap mode)."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    return _check(lib().conv_sep5_1pass(_ptr(d_in), _ptr(d_out), _taps(k), ctypes.byref(img),
                                        int(mode), _stream(stream)))


def conv_image_copy(d_in, d_out, img: conv_image | None = None, stream=None):
    """Copy an image with the library's streaming tile kernel (the copy-back
    step of the single pass with copy-back)."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    return _check(lib().conv_image_copy(_ptr(d_in), _ptr(d_out), ctypes.byref(img),
                                        _stream(stream)))


def conv_sepn_1pass(d_in, d_out, k, mode: int = CONV_1PASS_FUSED,
                    img: conv_image | None = None, stream=None):
    """Width-n separable single pass, n = len(k) odd in 1..9 (fused or direct)."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    taps, n = _taps_n(k)
    return _check(lib().conv_sepn_1pass(_ptr(d_in), _ptr(d_out), taps, n, ctypes.byref(img),
                                        int(mode), _stream(stream)))


def conv_sepn_2pass(d_in, d_out, k, d_tmp=None, img: conv_image | None = None, stream=None):
    """Width-n two-pass form, n = len(k) odd in 1..9."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    _check_workspace(d_tmp, img, 4)
    taps, n = _taps_n(k)
    return _check(lib().conv_sepn_2pass(_ptr(d_in), _ptr(d_out), _ptr(d_tmp), taps, n,
                                        ctypes.byref(img), _stream(stream)))


def conv_2d_direct(d_in, d_out, K, img: conv_image | None = None, stream=None):
    """Direct convolution with a full n x n kernel K (n odd in 1..9)."""
    if img is None:
        _same_layout(d_in, d_out)
        img = image_of(d_in)
    w, n = _kernel_nn(K)
    return _check(lib().conv_2d_direct(_ptr(d_in), _ptr(d_out), w, n, ctypes.byref(img),
                                       _stream(stream)))


def conv_pyr_down(d_in, d_out, k, in_img: conv_image | None = None,
                  out_img: conv_image | None = None, stream=None):
    """One pyramid level: width-5 blur, then every second row and column.
    d_out is [planes, ceil(rows/2), ceil(cols/2)] of d_in's dtype."""
    if in_img is None:
        in_img = image_of(d_in)
    if out_img is None:
        out_img = image_of(d_out)
    return _check(lib().conv_pyr_down(_ptr(d_in), ctypes.byref(in_img), _ptr(d_out),
                                      ctypes.byref(out_img), _taps(k), _stream(stream)))


def _batch_args(ins, outs, ks, imgs):
    n = len(ins)
    if len(outs) != n or len(ks) != n:
        raise ValueError("ins, outs and ks must have the same length")
    if imgs is None:
        for i, (a, b) in enumerate(zip(ins, outs)):
            _same_layout(a, b, f"output {i}")
        imgs = [image_of(t) for t in ins]
    imgs = list(imgs)
    pin = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value for t in ins])
    pout = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value for t in outs])
    flat = []
    for k in ks:
        flat.extend(float(v) for v in (k.tolist() if hasattr(k, "tolist") else k))
    if len(flat) != 5 * n:
        raise ValueError("each image needs 5 taps")
    kk = (ctypes.c_float * max(5 * n, 1))(*flat)
    ia = (conv_image * max(n, 1))(*imgs)
    return n, pin, pout, kk, ia


def conv_sep5_batch(ins: Sequence, outs: Sequence, ks: Sequence, imgs=None,
                    mode: int = CONV_1PASS_FUSED, stream=None):
    """Many images of different sizes in one launch."""
    n, pin, pout, kk, ia = _batch_args(ins, outs, ks, imgs)
    return _check(lib().conv_sep5_batch(n, pin, pout, kk, ia, int(mode), _stream(stream)))


class BatchPlan:
    """A batch bound to fixed buffers, replayed as a captured hipGraph."""

    def __init__(self, ins, outs, ks, imgs=None, mode: int = CONV_1PASS_FUSED):
        n, pin, pout, kk, ia = _batch_args(ins, outs, ks, imgs)
        h = ctypes.c_void_p()
        _check(lib().conv_batch_plan_create(n, pin, pout, kk, ia, int(mode), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        return _check(lib().conv_batch_plan_launch(self._h, _stream(stream)))

    def destroy(self):
        if self._h:
            lib().conv_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.destroy()
        except Exception:
            pass


def conv_batch_plan_create(ins, outs, ks, imgs=None, mode: int = CONV_1PASS_FUSED) -> BatchPlan:
    return BatchPlan(ins, outs, ks, imgs, mode)


def conv_get_tile_cfg(dtype: int, kind: int) -> conv_tile_cfg:
    c = conv_tile_cfg()
    _check(lib().conv_get_tile_cfg(int(dtype), int(kind), ctypes.byref(c)))
    return c


def conv_set_tile_cfg(dtype: int, kind: int, rows_per_tile: int, waves_per_wg: int,
                      persist_wgs_per_cu: int = 0, xcd_slabs: int = 0, pack_tail: int = 0):
    c = conv_tile_cfg(int(rows_per_tile), int(waves_per_wg), int(persist_wgs_per_cu),
                      int(xcd_slabs), int(pack_tail))
    return _check(lib().conv_set_tile_cfg(int(dtype), int(kind), ctypes.byref(c)))


def conv_get_tile_cfg_for(dtype: int, kind: int, footprint_bytes: int):
    """(configuration, tuned) that a call with this input + output byte count runs with."""
    c = conv_tile_cfg()
    t = ctypes.c_int32()
    _check(lib().conv_get_tile_cfg_for(int(dtype), int(kind), int(footprint_bytes),
                                       ctypes.byref(c), ctypes.byref(t)))
    return c, bool(t.value)


def conv_tune_save(path: str):
    return _check(lib().conv_tune_save(os.fsencode(path)))


def conv_tune_load(path: str):
    return _check(lib().conv_tune_load(os.fsencode(path)))


def conv_tune(kind: int, ins, outs, ks, imgs=None, reps: int = 5, stream=None):
    """Time every tile configuration on this workload; install the best for
    its size class and return (configuration, median ms)."""
    n, pin, pout, kk, ia = _batch_args(ins, outs, ks, imgs)
    best = conv_tile_cfg()
    ms = ctypes.c_float()
    _check(lib().conv_tune(int(kind), n, pin, pout, kk, ia, int(reps), _stream(stream),
                           ctypes.byref(best), ctypes.byref(ms)))
    return best, float(ms.value)


class Server:
    """Continuous-batching server (see conv_serve_* in the C header)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, n_streams: int = 4,
                 max_batch: int = 16, device: int = -1, max_batch_bytes: int = 0,
                 producer_wait: bool = True, queue_only: bool = True, launch_depth: int = 1):
        cfg = conv_serve_cfg(int(hbm_budget_bytes), int(max_slots), int(n_streams),
                             int(max_batch), int(device), int(max_batch_bytes),
                             int(bool(producer_wait)), int(bool(queue_only)), int(launch_depth))
        h = ctypes.c_void_p()
        _check(lib().conv_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, d_in, d_out, k, img: conv_image | None = None, stream=None) -> int:
        """Queue one request.  Work already enqueued on `stream` (default: torch's
        current stream) completes before the request's kernel starts."""
        if img is None:
            _same_layout(d_in, d_out)
            img = image_of(d_in)
        t = ctypes.c_uint64()
        _check(lib().conv_serve_submit(self._h, _ptr(d_in), _ptr(d_out), _taps(k),
                                       ctypes.byref(img), _stream(stream), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        """None while pending; the request's timestamps (dict) once done."""
        t = conv_req_times()
        st = lib().conv_serve_poll(self._h, int(ticket), ctypes.byref(t))
        if st == CONV_EAGAIN:
            return None
        _check(st)
        return t.as_dict()

    def drain(self):
        return _check(lib().conv_serve_drain(self._h))

    def stats(self) -> dict:
        st = conv_serve_stats()
        _check(lib().conv_serve_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def destroy(self):
        if self._h:
            _check(lib().conv_serve_destroy(self._h))
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.destroy()
        except Exception:
            pass


def conv_serve_create(hbm_budget_bytes: int, max_slots: int = 64, n_streams: int = 4,
                      max_batch: int = 16, device: int = -1, max_batch_bytes: int = 0,
                      producer_wait: bool = True, queue_only: bool = True,
                      launch_depth: int = 1) -> Server:
    return Server(hbm_budget_bytes, max_slots, n_streams, max_batch, device, max_batch_bytes,
                  producer_wait, queue_only, launch_depth)


def conv_serve_submit(srv: Server, d_in, d_out, k, img=None, stream=None) -> int:
    return srv.submit(d_in, d_out, k, img, stream)


def conv_serve_poll(srv: Server, ticket: int):
    return srv.poll(ticket)


def conv_serve_drain(srv: Server):
    return srv.drain()


def conv_serve_get_stats(srv: Server) -> dict:
    return srv.stats()


def conv_serve_destroy(srv: Server):
    return srv.destroy()


def conv_version() -> str:
    return lib().conv_version().decode()
