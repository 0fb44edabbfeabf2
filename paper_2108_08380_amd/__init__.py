"""BAD / HashSIFT describe-and-match on AMD MI355X (gfx950).

Thin Python binding over the C ABI in include/bdesc.h (libbdesc.so, built
in-tree by `python -m paper_2108_08380_amd.build`).  Every function here only
marshals torch tensors (device memory) and the current HIP stream into the C
call of the same name; all arithmetic runs in the library's HIP kernels.
There is no CPU fallback: without the built library every call raises.

Tensor conventions (all on one ROCm device, row stride free, unit column
stride):
  image        (H, W) uint8, or float32 for HashSIFT
  integral     (H+1, W+1) uint32
  keypoints    (n, 4) float32 rows (x, y, scale, angle)
  box pairs    (n_bits, 12) uint8 rows in the 12-byte bd_box_pair layout
  codes        (n, n_bits/64) uint64, bit j in word j/64 at position j%64
  knn          idx (n_q, k) int32, dist (n_q, k) uint32
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbdesc.so")

BD_OK, BD_EINVAL, BD_EUNSUPPORTED, BD_ENOMEM, BD_EDEVICE = 0, -1, -2, -3, -4
BD_DTYPE_U8, BD_DTYPE_F32, BD_DTYPE_F32_ROWPAIR = 0, 1, 2
BD_PREC_FP32, BD_PREC_BF16, BD_PREC_FP8 = 0, 1, 2
_PRECISIONS = {"fp32": BD_PREC_FP32, "bf16": BD_PREC_BF16, "fp8": BD_PREC_FP8}
DEFAULT_MARGIN = 1e-3
# train rows per split of the int8 MFMA k-NN engine (BD_BATCH_MFMA_MAX_ROWS)
MFMA_MAX_ROWS = 2048
# fixed device scratch of bd_match_hamming_knn_noalloc (BD_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 16 * 1024 * 1024

# Exported symbols of include/bdesc.h with their C signatures.
_P, _I32, _I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "bd_context_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int], ctypes.c_int),
    "bd_context_destroy": ([_P], ctypes.c_int),
    "bd_context_poll": ([_P, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "bd_last_error": ([], ctypes.c_char_p),
    "bd_version": ([], ctypes.c_char_p),
    "bd_build_integral": ([_P, _P, _I32, _I32, _I64, _P, _I64, _P], ctypes.c_int),
    "bd_bad_table_create": ([_P, _P, _I32, ctypes.POINTER(ctypes.c_void_p), _P], ctypes.c_int),
    "bd_bad_table_destroy": ([_P], ctypes.c_int),
    "bd_describe_bad_table": ([_P, _P, _I32, _I32, _I64, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "bd_keypoint_order": ([_P, _P, _I32, _I32, _I32, _P, _P], ctypes.c_int),
    "bd_build_integral_order": ([_P, _P, _I32, _I32, _I64, _P, _I64, _P, _I32, _P, _P], ctypes.c_int),
    "bd_prepare_view": ([_P, _P, _I32, _I32, _I64, _P, _I64, _P, _I32, _P, _P, _I64, _P, _I64, _P], ctypes.c_int),
    "bd_describe_bad": ([_P, _P, _I32, _I32, _I64, _P, _I32, _P, _P, _I32, _P, _P], ctypes.c_int),
    "bd_describe_hashsift": ([_P, _P, _I32, _I32, _I32, _I64, _P, _I32, _P, _P, _P, _I32, _I32, ctypes.c_float,
                              _P, _P, _P, _P, _P], ctypes.c_int),
    "bd_hashsift_features": ([_P, _P, _I32, _I32, _I32, _I64, _P, _I32, _P, _P, _P], ctypes.c_int),
    "bd_hashsift_project": ([_P, _P, _P, _I32, _P, _P, _I32, _I32, ctypes.c_float, _P, _P, _P, _P], ctypes.c_int),
    "bd_match_hamming_knn": ([_P, _P, _I32, _P, _I32, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "bd_match_hamming_knn_noalloc": ([_P, _P, _I32, _P, _I32, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "bd_match_mutual": ([_P, _P, _I32, _P, _I32, _I32, ctypes.c_float, _P, _P, _P, _P, _P], ctypes.c_int),
    "bd_find_threshold": ([_P, _P, _I32, _P, _P, ctypes.c_float, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "bd_select_features": ([_P, _P, _I32, _P, _I32, _P, _I32, _I32, ctypes.c_float, _P, _P, _P, _P, _P, _P],
                           ctypes.c_int),
    "bd_hashsift_patch_features": ([_P, _P, _I32, _P, _P], ctypes.c_int),
    "bd_relaxed_bad_fwd": ([_P, _P, _I32, _P, _P, _P, _P, _I32, ctypes.c_float, _P, _P, _P, _P], ctypes.c_int),
    "bd_relaxed_bad_bwd": ([_P, _P, _P, _P, _P, _I32, _I32, ctypes.c_float, _P, _P, _P, _P], ctypes.c_int),
    "bd_relaxed_hashsift_fwd": ([_P, _P, _I32, _P, _P, _I32, ctypes.c_float, _P, _P, _P], ctypes.c_int),
    "bd_relaxed_hashsift_bwd": ([_P, _P, _P, _P, _I32, _I32, ctypes.c_float, _P, _P, _P], ctypes.c_int),
    "bd_trl_hnm_fwd": ([_P, _P, _P, _I32, _I32, ctypes.c_float, _P, _P, _P, _P], ctypes.c_int),
    "bd_trl_hnm_bwd": ([_P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "bd_augment_patches": ([_P, _P, _I32, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "bd_hashsift_train_step": ([_P, _P, _I32, _P, _I32, _P, _P, _P, _P, _I32, _P, _I32, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, _P, _P], ctypes.c_int),
    "bd_batch_create": ([_P, _P, _I32, _P, _I32, _I32, _I32, _I32, ctypes.c_float, _I32,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "bd_batch_destroy": ([_P], ctypes.c_int),
    "bd_batch_run": ([_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _P], ctypes.c_int),
    "bd_batch_autotune": ([_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _P], ctypes.c_int),
    "bd_batch_default_tuning": ([_P], ctypes.c_int),
    "bd_batch_get_tuning": ([_P, _P], ctypes.c_int),
    "bd_batch_set_tuning": ([_P, _P], ctypes.c_int),
    "bd_batch_info": ([_P, _P, _P], ctypes.c_int),
}


class BatchImageRec(ctypes.Structure):
    """bd_batch_image."""
    _fields_ = [("img", ctypes.c_void_p), ("pitch", ctypes.c_int64), ("hs_img", ctypes.c_void_p),
                ("hs_pitch", ctypes.c_int64), ("hs_dtype", ctypes.c_int32), ("W", ctypes.c_int32),
                ("H", ctypes.c_int32), ("n_kp", ctypes.c_int32)]


class BatchMatchRec(ctypes.Structure):
    """bd_batch_match."""
    _fields_ = [("query_image", ctypes.c_int32), ("train_image", ctypes.c_int32)]


class BatchTuning(ctypes.Structure):
    """bd_batch_tuning; index 0 of the knn_* pairs is the BAD matcher, 1 the HashSIFT matcher."""
    _fields_ = [("order_blocks_per_cu", ctypes.c_int32), ("integral_blocks_per_cu", ctypes.c_int32),
                ("bad_blocks_per_cu", ctypes.c_int32), ("hist_blocks_per_cu", ctypes.c_int32),
                ("knn_qpl", ctypes.c_int32 * 2), ("knn_rows", ctypes.c_int32 * 2),
                ("knn_blocks_per_cu", ctypes.c_int32 * 2)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else int(v)
        return out


assert ctypes.sizeof(BatchImageRec) == 48 and ctypes.sizeof(BatchTuning) == 40


class BDError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


_lib = None
_lock = threading.Lock()
_contexts: dict = {}


def lib() -> ctypes.CDLL:
    """The loaded libbdesc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2108_08380_amd.build`")
                L = ctypes.CDLL(LIB_PATH)
                for name, (args, res) in SIGNATURES.items():
                    fn = getattr(L, name)
                    fn.argtypes = args
                    fn.restype = res
                _lib = L
    return _lib


def last_error() -> str:
    return lib().bd_last_error().decode()


def _check(rc: int) -> None:
    if rc != BD_OK:
        raise BDError(rc, last_error())


def context(device: int, stream=None) -> int:
    """The library context of (device, stream), created on first use.  Each
    stream gets its own context, hence its own workspace, so work enqueued on
    different streams never shares scratch memory."""
    key = (device, stream)
    ctx = _contexts.get(key)
    if ctx is None:
        with _lock:
            ctx = _contexts.get(key)
            if ctx is None:
                out = ctypes.c_void_p()
                _check(lib().bd_context_create(ctypes.byref(out), device))
                ctx = out.value
                _contexts[key] = ctx
    return ctx


def context_poll(device: int, stream=None) -> int:
    """bd_context_poll on the context of (device, stream): the number of invalid
    keypoints its describe calls met since the last poll (synchronizes)."""
    n = ctypes.c_uint64()
    _check(lib().bd_context_poll(context(device, stream), ctypes.byref(n)))
    return int(n.value)


def _torch():
    import torch
    return torch


def _device_and_stream(*tensors):
    torch = _torch()
    dev = tensors[0].device
    for t in tensors:
        if t is None:
            continue
        if t.device != dev or dev.type != "cuda":
            raise ValueError("all tensors must live on the same ROCm device")
    return dev.index, torch.cuda.current_stream(dev).cuda_stream


def _require(t, dtype, ndim, name):
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise ValueError(f"{name}: expected {ndim} dimensions, got {t.dim()}")
    if ndim >= 2 and t.stride(-1) != 1:
        raise ValueError(f"{name}: columns must be contiguous")


def _contig(t, name):
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


# --------------------------------------------------------------------------- marshalling helpers


def keypoints_tensor(kps: np.ndarray, device="cuda"):
    """(n,) structured keypoints or (n, 4) float32 array -> (n, 4) float32 device tensor."""
    torch = _torch()
    arr = np.ascontiguousarray(kps)
    if arr.dtype.names:
        arr = arr.view(np.float32).reshape(-1, 4)
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32).reshape(-1, 4)).to(device)


def pairs_tensor(pairs: np.ndarray, device="cuda"):
    """(n_bits,) structured box pairs (12-byte records) -> (n_bits, 12) uint8 device tensor."""
    torch = _torch()
    arr = np.ascontiguousarray(pairs)
    assert arr.dtype.itemsize == 12
    return torch.from_numpy(arr.view(np.uint8).reshape(-1, 12).copy()).to(device)


# --------------------------------------------------------------------------- entry points


def integral_buffer(H, W, device):
    """An (H+1, W+1) uint32 view whose rows start 16-byte aligned (row stride
    W+1 rounded up to a multiple of 4), the layout the integral-image kernel
    writes with full-width stores."""
    torch = _torch()
    pitch = (W + 1 + 3) // 4 * 4
    return torch.empty((H + 1, pitch), dtype=torch.uint32, device=device)[:, :W + 1]


def build_integral(img, out=None):
    """(H, W) uint8 image -> (H+1, W+1) uint32 integral image (bd_build_integral).
    Without `out`, the result is an integral_buffer view (padded rows)."""
    torch = _torch()
    _require(img, torch.uint8, 2, "img")
    H, W = img.shape
    if out is None:
        out = integral_buffer(H, W, img.device)
    _require(out, torch.uint32, 2, "out")
    dev, stream = _device_and_stream(img, out)
    _check(lib().bd_build_integral(context(dev, stream), img.data_ptr(), W, H, img.stride(0), out.data_ptr(),
                                   out.stride(0), stream))
    return out


def _order_arg(order, n):
    torch = _torch()
    if order is None:
        return None
    if order.dtype != torch.int32 or order.shape != (n,) or not order.is_contiguous():
        raise ValueError("order must be a contiguous (n_kp,) int32 tensor")
    return order.data_ptr()


def keypoint_order(kps, width: int, height: int, out=None):
    """Spatial processing order of keypoints (bd_keypoint_order) -> (n,) int32 permutation."""
    torch = _torch()
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    n = kps.shape[0]
    if out is None:
        out = torch.empty((n,), dtype=torch.int32, device=kps.device)
    dev, stream = _device_and_stream(kps, out)
    _check(lib().bd_keypoint_order(context(dev, stream), kps.data_ptr(), n, width, height, out.data_ptr(), stream))
    return out


def build_integral_order(img, kps, out=None, order=None):
    """Integral image and keypoint order of one view in one call
    (bd_build_integral_order) -> (ii, order), as build_integral and
    keypoint_order would return them."""
    torch = _torch()
    _require(img, torch.uint8, 2, "img")
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    H, W = img.shape
    n = kps.shape[0]
    if out is None:
        out = integral_buffer(H, W, img.device)
    _require(out, torch.uint32, 2, "out")
    if order is None:
        order = torch.empty((n,), dtype=torch.int32, device=img.device)
    dev, stream = _device_and_stream(img, kps, out, order)
    _check(lib().bd_build_integral_order(context(dev, stream), img.data_ptr(), W, H, img.stride(0), out.data_ptr(),
                                         out.stride(0), kps.data_ptr(), n, _order_arg(order, n), stream))
    return out, order


def prepare_view(img, kps, hs_img=None, out=None, order=None, pairs=None):
    """Integral image, keypoint order and (with a float32 hs_img) the row-pair
    copy of the HashSIFT image of one view in one call (bd_prepare_view)
    -> (ii, order, pairs); pairs is an (H, W, 2) float32 tensor that
    hashsift_features and describe_hashsift accept in place of hs_img."""
    torch = _torch()
    _require(img, torch.uint8, 2, "img")
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    H, W = img.shape
    n = kps.shape[0]
    if out is None:
        out = integral_buffer(H, W, img.device)
    _require(out, torch.uint32, 2, "out")
    if order is None:
        order = torch.empty((n,), dtype=torch.int32, device=img.device)
    hs_ptr, hs_pitch, pairs_ptr, pairs_pitch = None, 0, None, 0
    if hs_img is None and pairs is not None:
        raise ValueError("pairs is written from hs_img: pass both or neither")
    if hs_img is not None:
        _require(hs_img, torch.float32, 2, "hs_img")
        if tuple(hs_img.shape) != (H, W):
            raise ValueError("hs_img must have the shape of img")
        if pairs is None:
            pairs = torch.empty((H, W, 2), dtype=torch.float32, device=img.device)
        if _image_dtype(pairs) != BD_DTYPE_F32_ROWPAIR or tuple(pairs.shape) != (H, W, 2):
            raise ValueError("pairs must be an (H, W, 2) float32 tensor with contiguous pairs")
        hs_ptr, hs_pitch = hs_img.data_ptr(), hs_img.stride(0) * 4
        pairs_ptr, pairs_pitch = pairs.data_ptr(), pairs.stride(0) * 4
    dev, stream = _device_and_stream(img, kps, out, order, hs_img, pairs)
    _check(lib().bd_prepare_view(context(dev, stream), img.data_ptr(), W, H, img.stride(0), out.data_ptr(),
                                 out.stride(0), kps.data_ptr(), n, _order_arg(order, n), hs_ptr, hs_pitch, pairs_ptr,
                                 pairs_pitch, stream))
    return out, order, pairs


def describe_bad(ii, kps, pairs=None, n_bits: int | None = None, out=None, order=None, table=None):
    """BAD codes from an integral image (bd_describe_bad, or bd_describe_bad_table
    when a compiled BadTable is given instead of pairs)."""
    torch = _torch()
    _require(ii, torch.uint32, 2, "ii")
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    if table is not None:
        H, W = ii.shape[0] - 1, ii.shape[1] - 1
        n = kps.shape[0]
        if out is None:
            out = torch.empty((n, table.n_bits // 64), dtype=torch.uint64, device=ii.device)
        _contig(out, "out")
        dev, stream = _device_and_stream(ii, kps, out, order)
        _check(lib().bd_describe_bad_table(context(dev, stream), ii.data_ptr(), W, H, ii.stride(0), kps.data_ptr(), n,
                                           _order_arg(order, n), table._h, out.data_ptr(), stream))
        return out
    _contig(pairs, "pairs")
    if pairs.dtype != torch.uint8 or pairs.dim() != 2 or pairs.shape[1] != 12:
        raise TypeError("pairs must be an (n_bits, 12) uint8 tensor")
    n_bits = pairs.shape[0] if n_bits is None else n_bits
    if pairs.shape[0] < n_bits:
        raise ValueError("fewer box pairs than n_bits")
    H, W = ii.shape[0] - 1, ii.shape[1] - 1
    n = kps.shape[0]
    if out is None:
        out = torch.empty((n, n_bits // 64), dtype=torch.uint64, device=ii.device)
    _contig(out, "out")
    dev, stream = _device_and_stream(ii, kps, pairs, out, order)
    _check(lib().bd_describe_bad(context(dev, stream), ii.data_ptr(), W, H, ii.stride(0), kps.data_ptr(), n,
                                 _order_arg(order, n), pairs.data_ptr(), n_bits, out.data_ptr(), stream))
    return out


class BadTable:
    """A compiled BAD table (bd_bad_table_create): the pairs' distinct boxes in
    spatial order.  Use with describe_bad(..., table=...)."""

    def __init__(self, pairs, n_bits: int | None = None):
        torch = _torch()
        _contig(pairs, "pairs")
        if pairs.dtype != torch.uint8 or pairs.dim() != 2 or pairs.shape[1] != 12:
            raise TypeError("pairs must be an (n_bits, 12) uint8 tensor")
        self.n_bits = pairs.shape[0] if n_bits is None else n_bits
        if pairs.shape[0] < self.n_bits:
            raise ValueError("fewer box pairs than n_bits")
        dev, stream = _device_and_stream(pairs)
        self.device = dev
        out = ctypes.c_void_p()
        _check(lib().bd_bad_table_create(context(dev, stream), pairs.data_ptr(), self.n_bits, ctypes.byref(out),
                                         stream))
        self._h = out.value

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().bd_bad_table_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def describe_hashsift(img, kps, B, t, precision: str = "fp32", with_hist: bool = False,
                      with_resp: bool = False, out=None, order=None, margin: float = DEFAULT_MARGIN,
                      recheck_count=None):
    """HashSIFT codes (bd_describe_hashsift).  Returns codes, or (codes, hist, resp)
    when with_hist or with_resp is set (the unrequested ones are None).
    recheck_count: optional (1,) uint32 device tensor increased by the number of
    responses re-checked in FP32 (BF16/FP8 only)."""
    torch = _torch()
    dtype = _image_dtype(img)
    _require(img, img.dtype, 3 if dtype == BD_DTYPE_F32_ROWPAIR else 2, "img")
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    _require(B, torch.float32, 2, "B")
    _contig(B, "B")
    _contig(t, "t")
    n_bits = B.shape[0]
    if B.shape[1] != 128 or t.shape != (n_bits,) or t.dtype != torch.float32:
        raise ValueError("B must be (n_bits, 128) float32 and t (n_bits,) float32")
    H, W = img.shape[:2]
    n = kps.shape[0]
    if out is None:
        out = torch.empty((n, n_bits // 64), dtype=torch.uint64, device=img.device)
    hist = torch.empty((n, 128), dtype=torch.float32, device=img.device) if with_hist else None
    resp = torch.empty((n, n_bits), dtype=torch.float32, device=img.device) if with_resp else None
    dev, stream = _device_and_stream(img, kps, B, t, out, hist, resp, order, recheck_count)
    _check(lib().bd_describe_hashsift(context(dev, stream), img.data_ptr(), dtype, W, H, img.stride(0) * img.element_size(),
                                      kps.data_ptr(), n, _order_arg(order, n), B.data_ptr(), t.data_ptr(), n_bits,
                                      _PRECISIONS[precision], margin, out.data_ptr(),
                                      hist.data_ptr() if hist is not None else None,
                                      resp.data_ptr() if resp is not None else None,
                                      _counter_arg(recheck_count), stream))
    if with_hist or with_resp:
        return out, hist, resp
    return out


def _counter_arg(c):
    torch = _torch()
    if c is None:
        return None
    if c.dtype != torch.uint32 or c.numel() < 1:
        raise ValueError("recheck_count must be a uint32 device tensor")
    return c.data_ptr()


def _image_dtype(img):
    """Library dtype of a HashSIFT image: (H, W) uint8 or float32, or an
    (H, W, 2) float32 row-pair image from prepare_view."""
    torch = _torch()
    if img.dim() == 3:
        if img.dtype != torch.float32 or img.shape[2] != 2 or img.stride(2) != 1 or img.stride(1) != 2:
            raise TypeError("a row-pair image is an (H, W, 2) float32 tensor with contiguous pairs")
        return BD_DTYPE_F32_ROWPAIR
    if img.dtype == torch.uint8:
        return BD_DTYPE_U8
    if img.dtype == torch.float32:
        return BD_DTYPE_F32
    raise TypeError("img must be uint8 or float32")


def hashsift_features(img, kps, out=None, order=None):
    """(n, 128) float32 L2-normalized HashSIFT features (bd_hashsift_features)."""
    torch = _torch()
    dtype = _image_dtype(img)
    _require(img, img.dtype, 3 if dtype == BD_DTYPE_F32_ROWPAIR else 2, "img")
    _require(kps, torch.float32, 2, "kps")
    _contig(kps, "kps")
    H, W = img.shape[:2]
    n = kps.shape[0]
    if out is None:
        out = torch.empty((n, 128), dtype=torch.float32, device=img.device)
    _contig(out, "out")
    dev, stream = _device_and_stream(img, kps, out, order)
    _check(lib().bd_hashsift_features(context(dev, stream), img.data_ptr(), dtype, W, H, img.stride(0) * img.element_size(),
                                      kps.data_ptr(), n, _order_arg(order, n), out.data_ptr(), stream))
    return out


def hashsift_project(hist, B, t, kps=None, precision: str = "fp32", with_resp: bool = False, out=None,
                     margin: float = DEFAULT_MARGIN, recheck_count=None):
    """Codes (and optionally responses) of given features (bd_hashsift_project)."""
    torch = _torch()
    _require(hist, torch.float32, 2, "hist")
    _contig(hist, "hist")
    _require(B, torch.float32, 2, "B")
    _contig(B, "B")
    _contig(t, "t")
    n, n_bits = hist.shape[0], B.shape[0]
    if hist.shape[1] != 128 or B.shape[1] != 128 or t.shape != (n_bits,):
        raise ValueError("hist (n, 128), B (n_bits, 128), t (n_bits,)")
    if kps is not None:
        _contig(kps, "kps")
        if kps.shape[0] != n:
            raise ValueError("kps must have one row per feature row")
    if out is None:
        out = torch.empty((n, n_bits // 64), dtype=torch.uint64, device=hist.device)
    resp = torch.empty((n, n_bits), dtype=torch.float32, device=hist.device) if with_resp else None
    dev, stream = _device_and_stream(hist, B, t, out, kps, resp, recheck_count)
    _check(lib().bd_hashsift_project(context(dev, stream), hist.data_ptr(), kps.data_ptr() if kps is not None else None, n,
                                     B.data_ptr(), t.data_ptr(), n_bits, _PRECISIONS[precision], margin,
                                     out.data_ptr(), resp.data_ptr() if resp is not None else None,
                                     _counter_arg(recheck_count), stream))
    return (out, resp) if with_resp else out


def match_hamming_knn(query, train, k: int = 1, idx=None, dist=None):
    """Brute-force Hamming k-NN (bd_match_hamming_knn) -> (idx int32, dist uint32)."""
    torch = _torch()
    _require(query, torch.uint64, 2, "query")
    _require(train, torch.uint64, 2, "train")
    _contig(query, "query")
    _contig(train, "train")
    if query.shape[1] != train.shape[1]:
        raise ValueError("query and train codes differ in length")
    n_q, n_words = query.shape
    if idx is None:
        idx = torch.empty((n_q, k), dtype=torch.int32, device=query.device)
    if dist is None:
        dist = torch.empty((n_q, k), dtype=torch.uint32, device=query.device)
    dev, stream = _device_and_stream(query, train, idx, dist)
    _check(lib().bd_match_hamming_knn(context(dev, stream), query.data_ptr(), n_q, train.data_ptr(), train.shape[0],
                                      n_words, k, idx.data_ptr(), dist.data_ptr(), stream))
    return idx, dist


def match_hamming_knn_noalloc(query, train, idx, dist):
    """bd_match_hamming_knn_noalloc: the k-NN of match_hamming_knn with the
    library's fixed device scratch instead of the context workspace.  The
    caller supplies idx (n_q, k) int32 and dist (n_q, k) uint32; k is their
    column count.  The context of (device, stream) must already exist
    (context() creates it; creation is the only step that allocates)."""
    torch = _torch()
    _require(query, torch.uint64, 2, "query")
    _require(train, torch.uint64, 2, "train")
    _contig(query, "query")
    _contig(train, "train")
    _require(idx, torch.int32, 2, "idx")
    _require(dist, torch.uint32, 2, "dist")
    _contig(idx, "idx")
    _contig(dist, "dist")
    if query.shape[1] != train.shape[1]:
        raise ValueError("query and train codes differ in length")
    n_q, n_words = query.shape
    k = idx.shape[1]
    if idx.shape != (n_q, k) or dist.shape != (n_q, k):
        raise ValueError("idx and dist must both be (n_q, k)")
    dev, stream = _device_and_stream(query, train, idx, dist)
    ctx = _contexts.get((dev, stream))
    if ctx is None:
        raise RuntimeError("no library context for this device and stream; create it with context() first")
    _check(lib().bd_match_hamming_knn_noalloc(ctx, query.data_ptr(), n_q, train.data_ptr(), train.shape[0], n_words,
                                              k, idx.data_ptr(), dist.data_ptr(), stream))
    return idx, dist


def match_mutual(query, train, max_ratio: float = 0.0, with_ratio: bool = False, with_count: bool = False):
    """Mutual nearest neighbours with the distance-ratio filter (bd_match_mutual).
    Returns (match int32 (n_q,), dist uint32 (n_q,)) plus ratio float32 (n_q,) and
    count int32 (1,) when requested."""
    torch = _torch()
    _require(query, torch.uint64, 2, "query")
    _require(train, torch.uint64, 2, "train")
    _contig(query, "query")
    _contig(train, "train")
    if query.shape[1] != train.shape[1]:
        raise ValueError("query and train codes differ in length")
    n_q, n_words = query.shape
    match = torch.empty((n_q,), dtype=torch.int32, device=query.device)
    dist = torch.empty((n_q,), dtype=torch.uint32, device=query.device)
    ratio = torch.empty((n_q,), dtype=torch.float32, device=query.device) if with_ratio else None
    count = torch.empty((1,), dtype=torch.int32, device=query.device) if with_count else None
    dev, stream = _device_and_stream(query, train)
    _check(lib().bd_match_mutual(context(dev, stream), query.data_ptr(), n_q, train.data_ptr(), train.shape[0], n_words,
                                 max_ratio, match.data_ptr(), dist.data_ptr(),
                                 ratio.data_ptr() if ratio is not None else None,
                                 count.data_ptr() if count is not None else None, stream))
    out = (match, dist)
    if with_ratio:
        out += (ratio,)
    if with_count:
        out += (count,)
    return out


def find_threshold(patches, s_ap, s_an, tau: float, cands):
    """Alg. 2 threshold search for each candidate box pair (bd_find_threshold).
    patches (3n, 32, 32) uint8 (anchor, positive, negative interleaved), s_ap / s_an
    (n,) int32, cands (J, 12) uint8 box-pair records.  Returns (best_bin int32 (J,),
    best_theta float32 (J,), best_loss float64 (J,))."""
    torch = _torch()
    if patches.dtype != torch.uint8 or not patches.is_contiguous() or patches.numel() % 3072 != 0:
        raise ValueError("patches must be a contiguous (3n, 32, 32) uint8 tensor")
    n = patches.numel() // 3072
    for v, name in ((s_ap, "s_ap"), (s_an, "s_an")):
        if v.dtype != torch.int32 or tuple(v.shape) != (n,) or not v.is_contiguous():
            raise ValueError(f"{name} must be a contiguous ({n},) int32 tensor")
    _contig(cands, "cands")
    J = cands.shape[0]
    dev = patches.device
    best_bin = torch.empty((J,), dtype=torch.int32, device=dev)
    best_theta = torch.empty((J,), dtype=torch.float32, device=dev)
    best_loss = torch.empty((J,), dtype=torch.float64, device=dev)
    d, stream = _device_and_stream(patches, s_ap, s_an, cands)
    _check(lib().bd_find_threshold(context(d, stream), patches.data_ptr(), n, s_ap.data_ptr(), s_an.data_ptr(), tau,
                                   cands.data_ptr(), J, best_bin.data_ptr(), best_theta.data_ptr(),
                                   best_loss.data_ptr(), stream))
    return best_bin, best_theta, best_loss


def select_features(pool, samples, cands, tau: float = 1.0):
    """Greedy BAD feature selection, Alg. 1 (bd_select_features).
    pool (2P, 32, 32) uint8 (anchor, positive interleaved), samples (K, N) int32 pair
    indices, cands (K, J, 12) uint8 box-pair records.  Returns (table (K, 12) uint8
    box pairs with thresholds, chosen (K,) int32, chosen_bin (K,) int32, round_loss
    (K,) float64, pool_codes (2P, ceil(K/64)) uint64)."""
    torch = _torch()
    if pool.dtype != torch.uint8 or not pool.is_contiguous() or pool.numel() % 2048 != 0:
        raise ValueError("pool must be a contiguous (2P, 32, 32) uint8 tensor")
    n_pairs = pool.numel() // 2048
    if samples.dtype != torch.int32 or samples.dim() != 2 or not samples.is_contiguous():
        raise ValueError("samples must be a contiguous (K, N) int32 tensor")
    K, N = samples.shape
    if cands.dtype != torch.uint8 or cands.dim() != 3 or cands.shape[0] != K or cands.shape[2] != 12:
        raise ValueError("cands must be a (K, J, 12) uint8 tensor")
    _contig(cands, "cands")
    J = cands.shape[1]
    dev = pool.device
    table = torch.empty((K, 12), dtype=torch.uint8, device=dev)
    chosen = torch.empty((K,), dtype=torch.int32, device=dev)
    chosen_bin = torch.empty((K,), dtype=torch.int32, device=dev)
    loss = torch.empty((K,), dtype=torch.float64, device=dev)
    codes = torch.empty((2 * n_pairs, (K + 63) // 64), dtype=torch.uint64, device=dev)
    d, stream = _device_and_stream(pool, samples, cands)
    _check(lib().bd_select_features(context(d, stream), pool.data_ptr(), n_pairs, samples.data_ptr(), N, cands.data_ptr(),
                                    J, K, tau, table.data_ptr(), chosen.data_ptr(), chosen_bin.data_ptr(),
                                    loss.data_ptr(), codes.data_ptr(), stream))
    return table, chosen, chosen_bin, loss, codes


# --------------------------------------------------------------------------- differentiation extension


def _f32_contig(t, name, shape=None):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def hashsift_patch_features(patches, out=None):
    """(n, 128) HashSIFT features of (n, 32, 32) float32 patches (bd_hashsift_patch_features)."""
    torch = _torch()
    _f32_contig(patches, "patches")
    n = patches.shape[0]
    if patches.numel() != n * 1024:
        raise ValueError("patches must be (n, 32, 32)")
    if out is None:
        out = torch.empty((n, 128), dtype=torch.float32, device=patches.device)
    dev, stream = _device_and_stream(patches, out)
    _check(lib().bd_hashsift_patch_features(context(dev, stream), patches.data_ptr(), n, out.data_ptr(), stream))
    return out


def relaxed_bad_fwd(patches, pairs, w1, w2, theta, beta: float):
    """(D, m1, m2), each (n, K): relaxed BAD descriptors and the box means (bd_relaxed_bad_fwd)."""
    torch = _torch()
    _f32_contig(patches, "patches")
    n, K = patches.shape[0], pairs.shape[0]
    for v, name in ((w1, "w1"), (w2, "w2"), (theta, "theta")):
        _f32_contig(v, name, (K,))
    D = torch.empty((n, K), dtype=torch.float32, device=patches.device)
    m1, m2 = torch.empty_like(D), torch.empty_like(D)
    dev, stream = _device_and_stream(patches, pairs, w1, w2, theta)
    _check(lib().bd_relaxed_bad_fwd(context(dev, stream), patches.data_ptr(), n, pairs.data_ptr(), w1.data_ptr(),
                                    w2.data_ptr(), theta.data_ptr(), K, beta, D.data_ptr(), m1.data_ptr(),
                                    m2.data_ptr(), stream))
    return D, m1, m2


def relaxed_bad_bwd(gD, D, m1, m2, beta: float):
    """(g_w1, g_w2, g_theta) from dL/dD (bd_relaxed_bad_bwd)."""
    torch = _torch()
    n, K = D.shape
    for v, name in ((gD, "gD"), (D, "D"), (m1, "m1"), (m2, "m2")):
        _f32_contig(v, name, (n, K))
    g = [torch.empty((K,), dtype=torch.float32, device=D.device) for _ in range(3)]
    dev, stream = _device_and_stream(gD, D, m1, m2)
    _check(lib().bd_relaxed_bad_bwd(context(dev, stream), gD.data_ptr(), D.data_ptr(), m1.data_ptr(), m2.data_ptr(), n, K,
                                    beta, g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(), stream))
    return tuple(g)


def relaxed_hashsift_fwd(f, B, t, beta: float):
    """(rho, D), each (n, K), of the relaxed HashSIFT descriptor (bd_relaxed_hashsift_fwd)."""
    torch = _torch()
    n, K = f.shape[0], B.shape[0]
    _f32_contig(f, "f", (n, 128))
    _f32_contig(B, "B", (K, 128))
    _f32_contig(t, "t", (K,))
    rho = torch.empty((n, K), dtype=torch.float32, device=f.device)
    D = torch.empty_like(rho)
    dev, stream = _device_and_stream(f, B, t)
    _check(lib().bd_relaxed_hashsift_fwd(context(dev, stream), f.data_ptr(), n, B.data_ptr(), t.data_ptr(), K, beta,
                                         rho.data_ptr(), D.data_ptr(), stream))
    return rho, D


def relaxed_hashsift_bwd(gD, D, f, beta: float):
    """(gB, gt) from dL/dD (bd_relaxed_hashsift_bwd)."""
    torch = _torch()
    n, K = D.shape
    _f32_contig(gD, "gD", (n, K))
    _f32_contig(D, "D", (n, K))
    _f32_contig(f, "f", (n, 128))
    gB = torch.empty((K, 128), dtype=torch.float32, device=D.device)
    gt = torch.empty((K,), dtype=torch.float32, device=D.device)
    dev, stream = _device_and_stream(gD, D, f)
    _check(lib().bd_relaxed_hashsift_bwd(context(dev, stream), gD.data_ptr(), D.data_ptr(), f.data_ptr(), n, K, beta,
                                         gB.data_ptr(), gt.data_ptr(), stream))
    return gB, gt


def trl_hnm_fwd(A, P, tau: float):
    """(loss (1,), neg (n,) int32, hinge (n,)) of the hardest-negative triplet loss (bd_trl_hnm_fwd)."""
    torch = _torch()
    n, K = A.shape
    _f32_contig(A, "A", (n, K))
    _f32_contig(P, "P", (n, K))
    loss = torch.empty((1,), dtype=torch.float32, device=A.device)
    neg = torch.empty((n,), dtype=torch.int32, device=A.device)
    hinge = torch.empty((n,), dtype=torch.float32, device=A.device)
    dev, stream = _device_and_stream(A, P)
    _check(lib().bd_trl_hnm_fwd(context(dev, stream), A.data_ptr(), P.data_ptr(), n, K, tau, loss.data_ptr(), neg.data_ptr(),
                                hinge.data_ptr(), stream))
    return loss, neg, hinge


def trl_hnm_bwd(A, P, neg, hinge, grad_loss):
    """(gA, gP) for the upstream gradient grad_loss (a (1,) device tensor) (bd_trl_hnm_bwd)."""
    torch = _torch()
    n, K = A.shape
    gA, gP = torch.empty_like(A), torch.empty_like(P)
    grad_loss = _f32_contig(grad_loss.reshape(1).contiguous(), "grad_loss")
    dev, stream = _device_and_stream(A, P, neg, hinge, grad_loss)
    _check(lib().bd_trl_hnm_bwd(context(dev, stream), A.data_ptr(), P.data_ptr(), n, K, neg.data_ptr(), hinge.data_ptr(),
                                grad_loss.data_ptr(), gA.data_ptr(), gP.data_ptr(), stream))
    return gA, gP


# --------------------------------------------------------------------------- batching extension


class Batch:
    """A planned batch of images (bd_batch_create ... bd_batch_destroy).

    images:   list of (H, W) uint8 device tensors (integral image, BAD, and
              HashSIFT unless hs_images is given)
    n_kp:     keypoints per image; the flat keypoint array holds image 0's
              keypoints first, then image 1's, ...
    matches:  list of (query_image, train_image) index pairs
    hs_images: optional list of (H, W) uint8 or float32 tensors for HashSIFT
    (an entry of None: that image's u8 tensor); sources of both dtypes may be
    mixed.  The image tensors are kept alive by the batch."""

    def __init__(self, images, n_kp, matches=(), bad_bits: int = 512, hs_bits: int = 256,
                 precision: str = "fp32", margin: float = DEFAULT_MARGIN, k: int = 2, hs_images=None):
        torch = _torch()
        if len(images) != len(n_kp):
            raise ValueError("one keypoint count per image")
        if hs_images is not None and len(hs_images) != len(images):
            raise ValueError("one HashSIFT image per image")
        self._images = list(images)
        self._hs_images = list(hs_images) if hs_images is not None else None
        recs = (BatchImageRec * len(images))()
        for i, img in enumerate(images):
            _require(img, torch.uint8, 2, f"images[{i}]")
            H, W = img.shape
            recs[i].img, recs[i].pitch, recs[i].W, recs[i].H, recs[i].n_kp = img.data_ptr(), img.stride(0), W, H, int(n_kp[i])
            if hs_images is not None and hs_images[i] is not None:
                h = hs_images[i]
                if tuple(h.shape) != (H, W):
                    raise ValueError(f"hs_images[{i}] must match images[{i}] in shape")
                recs[i].hs_img = h.data_ptr()
                recs[i].hs_pitch = h.stride(0) * h.element_size()
                recs[i].hs_dtype = _image_dtype(h)
        mrecs = (BatchMatchRec * max(len(matches), 1))()
        for i, (q, t) in enumerate(matches):
            mrecs[i].query_image, mrecs[i].train_image = int(q), int(t)
        dev = images[0].device.index
        self.device = dev
        self.n_kp = [int(v) for v in n_kp]
        self.kp_offsets = np.concatenate([[0], np.cumsum(self.n_kp)]).astype(np.int64)
        self.matches = [(int(q), int(t)) for q, t in matches]
        self.match_offsets = np.concatenate([[0], np.cumsum([self.n_kp[q] for q, _ in self.matches])]).astype(np.int64)
        self.bad_bits, self.hs_bits, self.k = bad_bits, hs_bits, k
        out = ctypes.c_void_p()
        _check(lib().bd_batch_create(context(dev), recs, len(images), mrecs, len(matches), bad_bits, hs_bits,
                                     _PRECISIONS[precision], margin, k, ctypes.byref(out)))
        self._h = out.value

    @property
    def total_kp(self) -> int:
        return int(self.kp_offsets[-1])

    @property
    def match_rows(self) -> int:
        return int(self.match_offsets[-1])

    def allocate_outputs(self) -> dict:
        """Device output tensors of run(): codes per descriptor and idx/dist per matcher."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        out = {}
        if self.bad_bits:
            out["bad_codes"] = torch.empty((self.total_kp, self.bad_bits // 64), dtype=torch.uint64, device=dev)
            out["bad_idx"] = torch.empty((self.match_rows, self.k), dtype=torch.int32, device=dev)
            out["bad_dist"] = torch.empty((self.match_rows, self.k), dtype=torch.uint32, device=dev)
        if self.hs_bits:
            out["hs_codes"] = torch.empty((self.total_kp, self.hs_bits // 64), dtype=torch.uint64, device=dev)
            out["hs_idx"] = torch.empty((self.match_rows, self.k), dtype=torch.int32, device=dev)
            out["hs_dist"] = torch.empty((self.match_rows, self.k), dtype=torch.uint32, device=dev)
        return out

    def _args(self, kps, pairs, B, t, out):
        torch = _torch()
        _require(kps, torch.float32, 2, "kps")
        _contig(kps, "kps")
        if kps.shape[0] != self.total_kp:
            raise ValueError(f"kps must have {self.total_kp} rows")
        if self.bad_bits and (pairs is None or pairs.shape[0] < self.bad_bits):
            raise ValueError("need a BAD table of bad_bits pairs")
        if self.hs_bits and (B is None or tuple(B.shape) != (self.hs_bits, 128) or t is None):
            raise ValueError("need B (hs_bits, 128) and t (hs_bits,)")
        ptr = lambda x: x.data_ptr() if x is not None else None
        for v in out.values():
            _contig(v, "output")
        tensors = [kps, pairs, B, t] + list(out.values())
        _, stream = _device_and_stream(*[x for x in tensors if x is not None])
        return [kps.data_ptr(), ptr(pairs), ptr(B), ptr(t), ptr(out.get("bad_codes")), ptr(out.get("hs_codes")),
                ptr(out.get("bad_idx")), ptr(out.get("bad_dist")), ptr(out.get("hs_idx")),
                ptr(out.get("hs_dist"))], stream

    def run(self, kps, pairs=None, B=None, t=None, out=None, graph: bool = True) -> dict:
        """Describe and match the batch (bd_batch_run); returns the output dict."""
        out = self.allocate_outputs() if out is None else out
        args, stream = self._args(kps, pairs, B, t, out)
        _check(lib().bd_batch_run(self._h, *args, 1 if graph else 0, stream))
        return out

    def autotune(self, kps, pairs=None, B=None, t=None, out=None, reps: int = 3) -> dict:
        """Pick the fastest tuning on these inputs (bd_batch_autotune); returns the tuning."""
        out = self.allocate_outputs() if out is None else out
        args, stream = self._args(kps, pairs, B, t, out)
        _check(lib().bd_batch_autotune(self._h, *args, reps, stream))
        return self.tuning

    @property
    def tuning(self) -> dict:
        tn = BatchTuning()
        _check(lib().bd_batch_get_tuning(self._h, ctypes.byref(tn)))
        return tn.as_dict()

    @tuning.setter
    def tuning(self, values: dict) -> None:
        tn = BatchTuning()
        _check(lib().bd_batch_get_tuning(self._h, ctypes.byref(tn)))
        for name, v in values.items():
            cur = getattr(tn, name)
            if isinstance(cur, ctypes.Array):
                for i, x in enumerate(v):
                    cur[i] = int(x)
            else:
                setattr(tn, name, int(v))
        _check(lib().bd_batch_set_tuning(self._h, ctypes.byref(tn)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().bd_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_batch_tuning() -> dict:
    tn = BatchTuning()
    _check(lib().bd_batch_default_tuning(ctypes.byref(tn)))
    return tn.as_dict()


# --------------------------------------------------------------------------- HashSIFT training


def _pool_pairs(pool):
    torch = _torch()
    if pool.dtype != torch.float32 or not pool.is_contiguous() or pool.numel() % 2048 != 0:
        raise ValueError("pool must be a contiguous (2P, 32, 32) float32 tensor")
    return pool.numel() // 2048


def augment_patches(pool, batch, params, noise, out=None):
    """(2n, 32, 32) augmented patches of the batch's pairs (bd_augment_patches):
    anchors first, then positives; params (2n, 5), noise (2n, 32, 32) float32."""
    torch = _torch()
    n_pairs = _pool_pairs(pool)
    n = batch.shape[0]
    if batch.dtype != torch.int32 or not batch.is_contiguous():
        raise ValueError("batch must be a contiguous int32 tensor")
    _f32_contig(params, "params", (2 * n, 5))
    _f32_contig(noise, "noise")
    if noise.numel() != 2 * n * 1024:
        raise ValueError("noise must hold 2n x 1024 floats")
    if out is None:
        out = torch.empty((2 * n, 32, 32), dtype=torch.float32, device=pool.device)
    d, stream = _device_and_stream(pool, batch, params, noise, out)
    _check(lib().bd_augment_patches(context(d, stream), pool.data_ptr(), n_pairs, batch.data_ptr(), n, params.data_ptr(),
                                    noise.data_ptr(), out.data_ptr(), stream))
    return out


class HashSIFTTrainer:
    """Adam training of the HashSIFT projection (Sec. III-B) through
    bd_hashsift_train_step.  B (K, 128) starts from N(0, 0.25) unless given,
    t from zeros; lr 2e-4 as in the paper."""

    def __init__(self, n_bits: int = 512, device="cuda", B=None, t=None, lr: float = 2e-4, tau: float = 0.5,
                 beta: float = 1.0, seed: int = 0):
        torch = _torch()
        dev = torch.device(device)
        if B is None:
            g = torch.Generator().manual_seed(seed)
            B = torch.randn((n_bits, 128), generator=g, dtype=torch.float32) * 0.5  # variance 0.25
        self.B = B.to(dev).contiguous()
        self.t = (torch.zeros(n_bits) if t is None else t).to(dev, torch.float32).contiguous()
        self.state = torch.zeros(2 * n_bits * 128 + 2 * n_bits, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.n_bits, self.lr, self.tau, self.beta, self.step = n_bits, lr, tau, beta, 0

    def train_step(self, pool, batch, params, noise):
        """One iteration on the batch; returns the loss as a (1,) device tensor."""
        torch = _torch()
        n_pairs = _pool_pairs(pool)
        n = batch.shape[0]
        if batch.dtype != torch.int32 or not batch.is_contiguous():
            raise ValueError("batch must be a contiguous int32 tensor")
        _f32_contig(params, "params", (2 * n, 5))
        _f32_contig(noise, "noise")
        if noise.numel() != 2 * n * 1024:
            raise ValueError("noise must hold 2n x 1024 floats")
        self.step += 1
        d, stream = _device_and_stream(pool, batch, params, noise, self.B)
        _check(lib().bd_hashsift_train_step(context(d, stream), pool.data_ptr(), n_pairs, batch.data_ptr(), n,
                                            params.data_ptr(), noise.data_ptr(), self.B.data_ptr(),
                                            self.t.data_ptr(), self.n_bits, self.state.data_ptr(), self.step,
                                            self.lr, self.tau, self.beta, self.loss.data_ptr(), stream))
        return self.loss
