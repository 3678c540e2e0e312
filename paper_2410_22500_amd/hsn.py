"""Thin ctypes binding of libhsn.so (include/hsn.h).

Argument marshalling only: torch supplies device memory and the current
HIP stream; every step of the computation runs in the library's kernels.
There is no fallback: if libhsn.so is missing or fails to load, importing
this module raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_22500_amd.build`")
_lib = C.CDLL(LIB_PATH)

# status codes
OK, ERR_INVALID_ARG, ERR_SHAPE, ERR_UNSUPPORTED, ERR_OOM, ERR_DEVICE, ERR_NUMERIC = range(7)
U16, F32 = 0, 1
ALGO_MU, ALGO_ANLS, ALGO_HALS = 0, 1, 2
PREC_FP32, PREC_BF16 = 0, 1
INIT_USER, INIT_NNDSVDA, INIT_MLP, INIT_NNDSVD = 0, 1, 2, 3
MLP_IN, MLP_HIDDEN = 256, 128

(KERN_NMF_PASS, KERN_PROJECT, KERN_BACKPROJECT, KERN_NORMALIZE, KERN_NMF_PASS_BF16, KERN_MLP_ROWS,
 KERN_MLP_WGRAD, KERN_NNDSVD_GRAM, KERN_MLP_POOL, KERN_FBP_FILTER) = range(10)
KERN_COUNT = 10


class Dims(C.Structure):
    _fields_ = [("n_views", C.c_int64), ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("n_bins", C.c_int64)]


class NmfOpts(C.Structure):
    _fields_ = [("k", C.c_int), ("algo", C.c_int), ("precision", C.c_int), ("init", C.c_int),
                ("max_iter", C.c_int), ("check_every", C.c_int), ("polish_rounds", C.c_int),
                ("polish_algo", C.c_int), ("polish_bf16_rounds", C.c_int), ("rel_obj_tol", C.c_double),
                ("f_ref", C.c_double), ("mlp", C.c_void_p), ("mlp_pooled", C.c_void_p), ("bf16_bias", C.c_void_p),
                ("mlp_fallback_rel", C.c_double), ("anls_extrapolate", C.c_int)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class NmfStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("polish_done", C.c_int), ("objective", C.c_double), ("rel_obj", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int), ("history_len", C.c_int),
                ("ms", C.c_float), ("polish_bf16_done", C.c_int), ("fell_back", C.c_int)]


class NmfProblem(C.Structure):
    _fields_ = [("p", C.c_void_p), ("ldp", C.c_int64), ("n_p", C.c_int64), ("n_k", C.c_int64), ("k", C.c_int),
                ("V", C.c_void_p), ("D", C.c_void_p), ("f_ref", C.c_double), ("p_bf16", C.c_void_p),
                ("ldb", C.c_int64)]


BATCH_GRAPH, BATCH_AUTOTUNE = 1, 2


class Geom(C.Structure):
    _fields_ = [("n_views", C.c_int64), ("n_slices", C.c_int64), ("n_cols", C.c_int64), ("k", C.c_int),
                ("angles", C.POINTER(C.c_double))]


_P = C.c_void_p
_lib.hsn_create.argtypes = [C.POINTER(_P), C.c_int]
_lib.hsn_create.restype = C.c_int
_lib.hsn_destroy.argtypes = [_P]
_lib.hsn_destroy.restype = None
_lib.hsn_last_error.argtypes = [_P]
_lib.hsn_last_error.restype = C.c_char_p
_lib.hsn_version.restype = C.c_int
_lib.hsn_normalize.argtypes = [_P, C.POINTER(Dims), _P, C.c_int, _P, C.c_int, _P, C.c_float, C.c_int,
                               _P, C.c_int64, _P, C.c_int64, _P, _P, _P, _P]
_lib.hsn_normalize.restype = C.c_int
_lib.hsn_normalize_noalloc.argtypes = [_P, C.POINTER(Dims), _P, C.c_int, _P, C.c_int, _P, C.c_float, C.c_int,
                                       _P, C.c_int64, _P, C.c_int64, _P, _P, _P, _P]
_lib.hsn_normalize_noalloc.restype = C.c_int
_lib.hsn_normalize_pooled.argtypes = [_P, C.POINTER(Dims), _P, C.c_int, _P, C.c_int, _P, C.c_float, C.c_int,
                                      _P, C.c_int64, _P, C.c_int64, _P, _P, _P, _P, C.c_int, _P]
_lib.hsn_normalize_pooled.restype = C.c_int
_lib.hsn_subspace_nmf.argtypes = [_P, _P, C.c_int64, _P, C.c_int64, C.c_int64, C.c_int64, _P, _P,
                                  C.POINTER(NmfOpts), C.POINTER(NmfStats), _P]
_lib.hsn_subspace_nmf.restype = C.c_int
_lib.hsn_nmf_set_launch.argtypes = [_P, C.c_int]
_lib.hsn_nmf_set_launch.restype = C.c_int
_lib.hsn_subspace_nmf_batched.argtypes = [_P, C.c_int, C.POINTER(NmfProblem), C.POINTER(NmfOpts), C.c_int,
                                          C.POINTER(NmfStats), _P]
_lib.hsn_subspace_nmf_batched.restype = C.c_int
_lib.hsn_batched_plan_info.argtypes = [_P]
_lib.hsn_batched_plan_info.restype = C.c_char_p
_lib.hsn_project.argtypes = [_P, C.POINTER(Geom), _P, _P, C.c_float, C.c_float, _P]
_lib.hsn_project.restype = C.c_int
_lib.hsn_backproject.argtypes = [_P, C.POINTER(Geom), _P, _P, C.c_float, C.c_float, _P]
_lib.hsn_backproject.restype = C.c_int
_lib.hsn_cgls.argtypes = [_P, C.POINTER(Geom), _P, _P, C.c_int, _P, _P]
_lib.hsn_cgls.restype = C.c_int
_lib.hsn_fbp.argtypes = [_P, C.POINTER(Geom), _P, C.c_int64, _P, _P]
_lib.hsn_fbp.restype = C.c_int
_lib.hsn_fhr_step.argtypes = [_P, C.POINTER(Dims), _P, C.c_int, _P, C.c_int, C.c_float, _P, C.c_int64, _P,
                             C.c_int64, _P, _P, _P, C.POINTER(NmfOpts), C.POINTER(NmfStats), _P, C.c_int, _P,
                             C.c_int64, C.c_int64, C.c_int64, C.c_int64, _P, C.c_int64, _P]
_lib.hsn_fhr_step.restype = C.c_int
_lib.hsn_mbir.argtypes = [_P, C.POINTER(Geom), _P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                         C.c_double, C.c_int, C.c_int, _P]
_lib.hsn_mbir.restype = C.c_int
_lib.hsn_projector_set_launch.argtypes = [_P, C.c_int, C.c_int, C.c_int, C.c_int]
_lib.hsn_projector_set_launch.restype = C.c_int
_lib.hsn_projector_launch_info.argtypes = [_P, C.POINTER(Geom), C.POINTER(C.c_int)]
_lib.hsn_projector_launch_info.restype = C.c_int
_lib.hsn_rehydrate.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_int, C.c_int64, C.c_int64, C.c_int64,
                               C.c_int64, _P, C.c_int64, _P]
_lib.hsn_rehydrate.restype = C.c_int
_lib.hsn_mlp_n_params.argtypes = [C.c_int]
_lib.hsn_mlp_n_params.restype = C.c_int64
_lib.hsn_mlp_create.argtypes = [_P, C.POINTER(_P), C.c_int, C.c_int, _P]
_lib.hsn_mlp_create.restype = C.c_int
_lib.hsn_mlp_destroy.argtypes = [_P]
_lib.hsn_mlp_destroy.restype = None
_lib.hsn_mlp_get_params.argtypes = [_P, _P, _P]
_lib.hsn_mlp_get_params.restype = C.c_int
_lib.hsn_mlp_set_params.argtypes = [_P, _P, _P]
_lib.hsn_mlp_set_params.restype = C.c_int
_lib.hsn_mlp_k.argtypes = [_P]
_lib.hsn_mlp_k.restype = C.c_int
_lib.hsn_mlp_precision.argtypes = [_P]
_lib.hsn_mlp_precision.restype = C.c_int
_lib.hsn_mlp_pool.argtypes = [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int, _P, _P]
_lib.hsn_mlp_pool.restype = C.c_int
_lib.hsn_mlp_forward.argtypes = [_P, _P, _P, C.c_int64, _P, _P]
_lib.hsn_mlp_forward.restype = C.c_int
_lib.hsn_mlp_loss_grad.argtypes = [_P, _P, _P, _P, C.c_int64, _P, _P, _P]
_lib.hsn_mlp_loss_grad.restype = C.c_int
_lib.hsn_mlp_train.argtypes = [_P, _P, _P, _P, C.c_int64, C.POINTER(TrainOpts), _P, _P]
_lib.hsn_mlp_train.restype = C.c_int
_lib.hsn_mlp_infer.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_int64, _P, _P]
_lib.hsn_mlp_infer.restype = C.c_int
_lib.hsn_mlp_save.argtypes = [_P, _P, C.c_char_p]
_lib.hsn_mlp_save.restype = C.c_int
_lib.hsn_mlp_load.argtypes = [_P, C.POINTER(_P), C.c_char_p]
_lib.hsn_mlp_load.restype = C.c_int
_lib.hsn_canonicalize.argtypes = [_P, _P, C.c_int64, _P, C.c_int64, C.c_int, _P, _P]
_lib.hsn_canonicalize.restype = C.c_int
_lib.hsn_fmd.argtypes = [_P, _P, C.c_int64, C.c_int, _P, C.c_int, _P, C.c_int64, _P, _P, _P, _P]
_lib.hsn_fmd.restype = C.c_int
_lib.hsn_profile_enable.argtypes = [_P, C.c_int]
_lib.hsn_profile_enable.restype = C.c_int
_lib.hsn_profile_read.argtypes = [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
_lib.hsn_profile_read.restype = C.c_int


class HsnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hsn status {status}: {msg}")
        self.status = status


_ctx = {}


def context(device: int = 0):
    if device not in _ctx:
        h = _P()
        st = _lib.hsn_create(C.byref(h), device)
        if st != OK:
            raise HsnError(st, f"hsn_create(device={device}) failed")
        _ctx[device] = h
    return _ctx[device]


def _check(st: int, ctx) -> None:
    if st != OK:
        raise HsnError(st, _lib.hsn_last_error(ctx).decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else _P(t.data_ptr())


def _stream(dev) -> _P:
    return _P(torch.cuda.current_stream(dev).cuda_stream)


def _dev(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("hsn: tensors must live on a GPU")
    return t.device.index or 0


_U16 = (torch.int16, torch.uint16)


def _need(t, name: str, dtype, shape=None, layout: str = "contiguous", device=None, extent=None):
    """Reject, before any library call, a tensor the kernels would misread:
    wrong dtype, a shape that disagrees with the other arguments (None in
    `shape` matches any size), a layout the kernels do not index (layout
    "contiguous"; "rows": 2-D with unit column stride and a row pitch of at
    least its width, e.g. p[:, :n_k]; "inner": unit last-dimension stride),
    storage shorter than `extent` elements from the tensor's first element,
    or memory on another device than `device`.  Checked in that order; the
    wrappers then check (_dev) that the memory is on a GPU."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"hsn: {name} must be a torch.Tensor, got {type(t).__name__}")
    dts = dtype if isinstance(dtype, tuple) else (dtype,)
    if t.dtype not in dts:
        raise ValueError(f"hsn: {name} must have dtype {' or '.join(str(d) for d in dts)}, got {t.dtype}")
    if shape is not None and (t.dim() != len(shape) or any(s is not None and a != s for a, s in zip(t.shape, shape))):
        raise ValueError(f"hsn: {name} must have shape {tuple('*' if s is None else s for s in shape)}, "
                         f"got {tuple(t.shape)}")
    if layout == "contiguous" and not t.is_contiguous():
        raise ValueError(f"hsn: {name} must be contiguous (got strides {t.stride()})")
    if layout == "rows" and (t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.stride(0) < t.shape[1]):
        raise ValueError(f"hsn: {name} must be a 2-D array of rows with unit column stride (got strides {t.stride()})")
    if layout == "inner" and t.dim() > 0 and t.shape[-1] > 1 and t.stride(-1) != 1:
        raise ValueError(f"hsn: {name} needs a unit stride in its last dimension (got strides {t.stride()})")
    if extent is not None and t.untyped_storage().nbytes() // t.element_size() - t.storage_offset() < extent:
        raise ValueError(f"hsn: {name} holds fewer than the {extent} elements the call reads")
    if device is not None and t.device != device:
        raise ValueError(f"hsn: {name} is on {t.device}, the call's other tensors on {device}")
    return t


def _opt(t, *a, **kw):
    return None if t is None else _need(t, *a, **kw)


def _geom(n_views, n_slices, n_cols, k, angles):
    g = Geom(n_views, n_slices, n_cols, k, None)
    keep = None
    if angles is not None:
        keep = (C.c_double * n_views)(*[float(a) for a in angles])
        g.angles = C.cast(keep, C.POINTER(C.c_double))
    return g, keep


def round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def _check_counts(y, yo, bg_mask=None):
    _need(y, "y", _U16 + (torch.float32,), shape=(None, None, None, None))
    n_v, n_r, n_c, n_k = y.shape
    _need(yo, "y_open", _U16 + (torch.float32,), shape=(n_r, n_c, n_k), device=y.device)
    _opt(bg_mask, "bg_mask", torch.uint8, shape=(n_r, n_c), device=y.device)


def hsn_normalize(y: torch.Tensor, yo: torch.Tensor, bg_mask: Optional[torch.Tensor] = None,
                  count_floor: float = 1.0, clip: bool = True, want_f32: bool = True, want_bf16: bool = False,
                  want_offset: bool = False, ldp: Optional[int] = None, ldb: Optional[int] = None,
                  want_bias: bool = False):
    """y [N_v][N_r][N_c][N_k] (uint16 as int16/uint16 bits or float32), yo [N_r][N_c][N_k].
    Returns (p [N_p][ldp] f32 or None, p_bf16 [N_p][ldb] int16 bits or None, b or None, sumsq f64 scalar);
    with want_bias (needs want_bf16) a fifth item, the f64 scalar -||p - p_bf16||^2."""
    _check_counts(y, yo, bg_mask)
    dev = _dev(y)
    ctx = context(dev)
    n_v, n_r, n_c, n_k = y.shape
    dims = Dims(n_v, n_r, n_c, n_k)
    yd = F32 if y.dtype == torch.float32 else U16
    od = F32 if yo.dtype == torch.float32 else U16
    n_p = n_v * n_r * n_c
    ldp = ldp or round_up(n_k, 4)
    ldb = ldb or round_up(n_k, 32)
    p = torch.empty((n_p, ldp), dtype=torch.float32, device=y.device) if want_f32 else None
    pb = torch.empty((n_p, ldb), dtype=torch.int16, device=y.device) if want_bf16 else None
    b = torch.empty((n_v, n_k), dtype=torch.float32, device=y.device) if (want_offset and bg_mask is not None) else None
    ss = torch.empty((), dtype=torch.float64, device=y.device)
    bias = torch.empty((), dtype=torch.float64, device=y.device) if want_bias else None
    _check(_lib.hsn_normalize(ctx, C.byref(dims), _ptr(y), yd, _ptr(yo), od, _ptr(bg_mask), float(count_floor),
                              int(clip), _ptr(p), ldp, _ptr(pb), ldb, _ptr(b), _ptr(ss), _ptr(bias), _stream(dev)), ctx)
    return (p, pb, b, ss, bias) if want_bias else (p, pb, b, ss)


def hsn_normalize_noalloc(y: torch.Tensor, yo: torch.Tensor, p: Optional[torch.Tensor] = None,
                          p_bf16: Optional[torch.Tensor] = None, bg_mask: Optional[torch.Tensor] = None,
                          offset_b: Optional[torch.Tensor] = None, sumsq: Optional[torch.Tensor] = None,
                          bf16_bias: Optional[torch.Tensor] = None, count_floor: float = 1.0,
                          clip: bool = True) -> None:
    """hsn_normalize into caller-owned outputs (p [N_p][ldp] f32, p_bf16 [N_p][ldb] int16 bits, offset_b
    [N_v][N_k] f32 (required with bg_mask), sumsq and bf16_bias f64 scalars); the library allocates
    nothing for the call."""
    _check_counts(y, yo, bg_mask)
    n_v, n_r, n_c, n_k = y.shape
    n_p = n_v * n_r * n_c
    _opt(p, "p", torch.float32, shape=(n_p, None), layout="rows", device=y.device)
    _opt(p_bf16, "p_bf16", _U16, shape=(n_p, None), layout="rows", device=y.device)
    _opt(offset_b, "offset_b", torch.float32, shape=(n_v, n_k), device=y.device)
    _opt(sumsq, "sumsq", torch.float64, shape=(), device=y.device)
    _opt(bf16_bias, "bf16_bias", torch.float64, shape=(), device=y.device)
    dev = _dev(y)
    ctx = context(dev)
    dims = Dims(n_v, n_r, n_c, n_k)
    yd = F32 if y.dtype == torch.float32 else U16
    od = F32 if yo.dtype == torch.float32 else U16
    _check(_lib.hsn_normalize_noalloc(ctx, C.byref(dims), _ptr(y), yd, _ptr(yo), od, _ptr(bg_mask),
                                      float(count_floor), int(clip), _ptr(p), p.stride(0) if p is not None else 0,
                                      _ptr(p_bf16), p_bf16.stride(0) if p_bf16 is not None else 0, _ptr(offset_b),
                                      _ptr(sumsq), _ptr(bf16_bias), _stream(dev)), ctx)


def hsn_normalize_pooled(y: torch.Tensor, yo: torch.Tensor, pooled_precision: int, bg_mask: Optional[torch.Tensor] = None,
                         count_floor: float = 1.0, clip: bool = True, want_f32: bool = True, want_bf16: bool = False,
                         want_offset: bool = False, ldp: Optional[int] = None, ldb: Optional[int] = None,
                         want_bias: bool = False):
    """hsn_normalize plus the learned start's pooled input [N_p][256] (bfloat16 bits as int16 for
    PREC_BF16, float32 for PREC_FP32).  Returns (p, p_bf16, pooled, b, sumsq), plus the bias
    -||p - p_bf16||^2 with want_bias."""
    _check_counts(y, yo, bg_mask)
    dev = _dev(y)
    ctx = context(dev)
    n_v, n_r, n_c, n_k = y.shape
    dims = Dims(n_v, n_r, n_c, n_k)
    yd = F32 if y.dtype == torch.float32 else U16
    od = F32 if yo.dtype == torch.float32 else U16
    n_p = n_v * n_r * n_c
    ldp = ldp or round_up(n_k, 4)
    ldb = ldb or round_up(n_k, 32)
    p = torch.empty((n_p, ldp), dtype=torch.float32, device=y.device) if want_f32 else None
    pb = torch.empty((n_p, ldb), dtype=torch.int16, device=y.device) if want_bf16 else None
    pooled = torch.empty((n_p, 256), dtype=torch.int16 if pooled_precision == PREC_BF16 else torch.float32,
                         device=y.device)
    b = torch.empty((n_v, n_k), dtype=torch.float32, device=y.device) if (want_offset and bg_mask is not None) else None
    ss = torch.empty((), dtype=torch.float64, device=y.device)
    bias = torch.empty((), dtype=torch.float64, device=y.device) if want_bias else None
    _check(_lib.hsn_normalize_pooled(ctx, C.byref(dims), _ptr(y), yd, _ptr(yo), od, _ptr(bg_mask), float(count_floor),
                                     int(clip), _ptr(p), ldp, _ptr(pb), ldb, _ptr(b), _ptr(ss), _ptr(bias),
                                     _ptr(pooled), int(pooled_precision), _stream(dev)), ctx)
    return (p, pb, pooled, b, ss, bias) if want_bias else (p, pb, pooled, b, ss)


def hsn_subspace_nmf(p: Optional[torch.Tensor], p_bf16: Optional[torch.Tensor], n_k: int, V: torch.Tensor,
                     D: torch.Tensor, algo: int = ALGO_MU, precision: int = PREC_FP32, max_iter: int = 100,
                     check_every: int = 10, polish_rounds: int = 0, polish_algo: int = ALGO_ANLS,
                     polish_bf16_rounds: int = 0, rel_obj_tol: float = 0.0, f_ref: float = 0.0,
                     init: int = INIT_USER, mlp: Optional["Mlp"] = None, history_cap: int = 4096,
                     mlp_pooled: Optional[torch.Tensor] = None, bf16_bias: Optional[torch.Tensor] = None,
                     mlp_fallback_rel: float = 0.0, anls_extrapolate: bool = False) -> dict:
    """Runs eq. (4) in place on V [N_p][K] and D [N_k][K] (float32, device).  bf16_bias: the f64
    device scalar -||p - p_bf16||^2 (hsn_normalize want_bias) for the stop test of the
    polish rounds on p_bf16.  mlp_fallback_rel > 0: a learned start whose first objective is
    further than this above f_ref is replaced by NNDSVDa (stats fell_back)."""
    _need(V, "V", torch.float32, shape=(None, None))
    n_p, k = V.shape
    _need(D, "D", torch.float32, shape=(n_k, k), device=V.device)
    _opt(p, "p", torch.float32, shape=(n_p, None), layout="rows", device=V.device)
    _opt(p_bf16, "p_bf16", _U16, shape=(n_p, None), layout="rows", device=V.device)
    if mlp_pooled is not None:
        _need(mlp_pooled, "mlp_pooled", mlp.x_dtype if mlp is not None else (torch.int16, torch.float32),
              shape=(n_p, MLP_IN), device=V.device)
    if p is not None and p.shape[1] < n_k or p_bf16 is not None and p_bf16.shape[1] < n_k:
        raise ValueError(f"hsn: p and p_bf16 rows must hold n_k = {n_k} bins")
    dev = _dev(V)
    ctx = context(dev)
    _opt(bf16_bias, "bf16_bias", torch.float64, shape=(), device=V.device)
    opts = NmfOpts(k, algo, precision, init, max_iter, check_every, polish_rounds, polish_algo,
                   polish_bf16_rounds, rel_obj_tol, f_ref, mlp.handle if mlp is not None else None,
                   _ptr(mlp_pooled), _ptr(bf16_bias), float(mlp_fallback_rel), int(bool(anls_extrapolate)))
    hist = (C.c_double * max(history_cap, 1))()
    stats = NmfStats(0, 0, 0.0, 0.0, C.cast(hist, C.POINTER(C.c_double)), history_cap, 0, 0.0, 0, 0)
    ldp = p.stride(0) if p is not None else 0
    ldb = p_bf16.stride(0) if p_bf16 is not None else 0
    _check(_lib.hsn_subspace_nmf(ctx, _ptr(p), ldp, _ptr(p_bf16), ldb, n_p, n_k, _ptr(V), _ptr(D), C.byref(opts),
                                 C.byref(stats), _stream(dev)), ctx)
    return _stats(stats, hist)


def _stats(s, hist) -> dict:
    return dict(iters=s.iters, polish_done=s.polish_done, polish_bf16_done=s.polish_bf16_done, objective=s.objective,
                rel_obj=s.rel_obj, history=[hist[i] for i in range(s.history_len)], ms=s.ms,
                fell_back=bool(s.fell_back))


def hsn_nmf_set_launch(anls_passes: int = 0, device: int = 0) -> None:
    """Form of the ANLS rounds: 0 or 1 = one fused pass (default), 2 = N_V pass, row solves, N_D pass."""
    ctx = context(device)
    _check(_lib.hsn_nmf_set_launch(ctx, int(anls_passes)), ctx)


def hsn_subspace_nmf_batched(problems, max_iter: int = 100, check_every: int = 10, polish_rounds: int = 0,
                             rel_obj_tol: float = 0.0, flags: int = BATCH_GRAPH, history_cap: int = 4096,
                             precision: int = PREC_FP32):
    """problems: list of (p [N_p][ldp] f32, n_k, V [N_p][K], D [N_k][K], f_ref) or, with
    precision=PREC_BF16, (p, n_k, V, D, f_ref, p_bf16 [N_p][ldb] int16 bits); V and D in place.
    MU bulk (float32 or bfloat16 MFMA) then float32 ANLS polish, one launch per phase and kernel
    shape over all instances."""
    if not problems:
        raise ValueError("hsn: no problems")
    bf16 = precision == PREC_BF16 and max_iter > 0
    dev0 = problems[0][2].device if isinstance(problems[0][2], torch.Tensor) else None
    for i, prob in enumerate(problems):
        p, n_k, V, D = prob[:4]
        _need(V, f"problems[{i}].V", torch.float32, shape=(None, None), device=dev0)
        _need(D, f"problems[{i}].D", torch.float32, shape=(n_k, V.shape[1]), device=dev0)
        _need(p, f"problems[{i}].p", torch.float32, shape=(V.shape[0], None), layout="rows", device=dev0)
        if p.shape[1] < n_k:
            raise ValueError(f"hsn: problems[{i}].p rows must hold n_k = {n_k} bins")
        if bf16:
            if len(prob) < 6 or prob[5] is None:
                raise ValueError(f"hsn: problems[{i}]: the bfloat16 bulk needs p_bf16 (sixth item)")
            _need(prob[5], f"problems[{i}].p_bf16", _U16, shape=(V.shape[0], None), layout="rows", device=dev0)
            if prob[5].shape[1] < n_k:
                raise ValueError(f"hsn: problems[{i}].p_bf16 rows must hold n_k = {n_k} bins")
    dev = _dev(problems[0][2])
    ctx = context(dev)
    n = len(problems)
    arr = (NmfProblem * n)()
    for i, prob in enumerate(problems):
        p, n_k, V, D, f_ref = prob[:5]
        pb = prob[5] if bf16 else None
        arr[i] = NmfProblem(p.data_ptr(), p.stride(0), V.shape[0], n_k, V.shape[1], V.data_ptr(), D.data_ptr(),
                            float(f_ref or 0.0), _ptr(pb), pb.stride(0) if pb is not None else 0)
    opts = NmfOpts(1, ALGO_MU, precision, INIT_USER, max_iter, check_every, polish_rounds, ALGO_ANLS, 0,
                   rel_obj_tol, 0.0, None, None, None)
    hists = [(C.c_double * max(history_cap, 1))() for _ in range(n)]
    stats = (NmfStats * n)()
    for i in range(n):
        stats[i] = NmfStats(0, 0, 0.0, 0.0, C.cast(hists[i], C.POINTER(C.c_double)), history_cap, 0, 0.0, 0, 0)
    _check(_lib.hsn_subspace_nmf_batched(ctx, n, arr, C.byref(opts), flags, stats, _stream(dev)), ctx)
    return [_stats(s, hists[i]) for i, s in enumerate(stats)]


def hsn_batched_plan_info(device: int = 0) -> str:
    return _lib.hsn_batched_plan_info(context(device)).decode()


def hsn_project(x: torch.Tensor, n_views: int, angles: Optional[Sequence[float]] = None, alpha: float = 1.0,
                beta: float = 0.0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x [N_r][N][N][K] -> s [N_v][N_r][N][K]."""
    _need(x, "x", torch.float32, shape=(None, None, None, None))
    n_r, n, _, k = x.shape
    _need(x, "x", torch.float32, shape=(n_r, n, n, k))
    _opt(out, "out", torch.float32, shape=(n_views, n_r, n, k), device=x.device)
    dev = _dev(x)
    ctx = context(dev)
    g, keep = _geom(n_views, n_r, n, k, angles)
    if out is None:
        out = torch.empty((n_views, n_r, n, k), dtype=torch.float32, device=x.device)
    _check(_lib.hsn_project(ctx, C.byref(g), _ptr(x), _ptr(out), alpha, beta, _stream(dev)), ctx)
    return out


def hsn_backproject(s: torch.Tensor, angles: Optional[Sequence[float]] = None, alpha: float = 1.0, beta: float = 0.0,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """s [N_v][N_r][N][K] -> x [N_r][N][N][K]."""
    _need(s, "s", torch.float32, shape=(None, None, None, None))
    n_v, n_r, n, k = s.shape
    _opt(out, "out", torch.float32, shape=(n_r, n, n, k), device=s.device)
    dev = _dev(s)
    ctx = context(dev)
    g, keep = _geom(n_v, n_r, n, k, angles)
    if out is None:
        out = torch.empty((n_r, n, n, k), dtype=torch.float32, device=s.device)
    _check(_lib.hsn_backproject(ctx, C.byref(g), _ptr(s), _ptr(out), alpha, beta, _stream(dev)), ctx)
    return out


def hsn_projector_set_launch(views: int = 0, split: int = 0, voxels: int = 0, threads: int = 0,
                             device: int = 0) -> None:
    """Projector launch shape (A: views per block, ray-set copies per block; A^T: voxels per
    thread, threads per block); 0 = automatic, views / voxels -1 = gather kernels."""
    ctx = context(device)
    _check(_lib.hsn_projector_set_launch(ctx, int(views), int(split), int(voxels), int(threads)), ctx)


def hsn_projector_launch_info(n_views: int, n_slices: int, n: int, k: int,
                              angles: Optional[Sequence[float]] = None, device: int = 0):
    """(views, split, voxels, threads) the projector would use; 0 = gather kernel."""
    ctx = context(device)
    g, keep = _geom(n_views, n_slices, n, k, angles)
    out = (C.c_int * 4)()
    _check(_lib.hsn_projector_launch_info(ctx, C.byref(g), out), ctx)
    return tuple(out)


def hsn_cgls(sino: torch.Tensor, n_iter: int, angles: Optional[Sequence[float]] = None, resid: bool = False):
    """Per-channel CGLS from x = 0: sino [N_v][N_r][N][K] -> x [N_r][N][N][K] (and residual norms)."""
    _need(sino, "sino", torch.float32, shape=(None, None, None, None))
    dev = _dev(sino)
    ctx = context(dev)
    n_v, n_r, n, k = sino.shape
    g, keep = _geom(n_v, n_r, n, k, angles)
    x = torch.empty((n_r, n, n, k), dtype=torch.float32, device=sino.device)
    rh = torch.empty((n_iter + 1, k), dtype=torch.float64, device=sino.device) if resid else None
    _check(_lib.hsn_cgls(ctx, C.byref(g), _ptr(sino), _ptr(x), n_iter, _ptr(rh), _stream(dev)), ctx)
    return (x, rh) if resid else x


def hsn_fhr_step(y: torch.Tensor, yo: torch.Tensor, V: torch.Tensor, D: torch.Tensor, cgls_iters: int,
                 vox=None, bins=None, angles: Optional[Sequence[float]] = None, count_floor: float = 1.0,
                 bufs: Optional[dict] = None, algo: int = ALGO_MU, precision: int = PREC_FP32, max_iter: int = 100,
                 check_every: int = 10, polish_rounds: int = 0, polish_algo: int = ALGO_ANLS,
                 polish_bf16_rounds: int = 0, rel_obj_tol: float = 0.0, f_ref: float = 0.0, init: int = INIT_USER,
                 mlp: Optional["Mlp"] = None, history_cap: int = 4096, mlp_fallback_rel: float = 0.0,
                 anls_extrapolate: bool = False):
    """The whole FHR path of one scan in one C call: counts y [N_v][N_r][N_c][N_k] and y^o (uint16 bits
    as int16) -> V, D in place, x [N_r][N_c][N_c][K], and x^h over vox x bins (None if vox is None).
    bufs: optional dict that keeps the intermediates (p, pooled) and outputs (x, xh) between calls."""
    _check_counts(y, yo)
    n_v, n_r, n_c, n_k = y.shape
    _need(V, "V", torch.float32, shape=(n_v * n_r * n_c, None), device=y.device)
    _need(D, "D", torch.float32, shape=(n_k, V.shape[1]), device=y.device)
    dev = _dev(y)
    ctx = context(dev)
    n_p, k = V.shape
    dims = Dims(n_v, n_r, n_c, n_k)
    bufs = {} if bufs is None else bufs
    ldp = round_up(n_k, 4)
    if "p" not in bufs:
        bufs["p"] = torch.empty((n_p, ldp), dtype=torch.float32, device=y.device)
    ldb = round_up(n_k, 32)
    uses_bf16 = polish_bf16_rounds > 0 or (precision == PREC_BF16 and max_iter > 0)
    if uses_bf16 and "p_bf16" not in bufs:
        bufs["p_bf16"] = torch.empty((n_p, ldb), dtype=torch.int16, device=y.device)
    pb = bufs.get("p_bf16") if uses_bf16 else None
    learned = init == INIT_MLP
    if learned and mlp is not None and "pooled" not in bufs:
        bufs["pooled"] = torch.empty((n_p, MLP_IN), dtype=mlp.x_dtype, device=y.device)
    if "x" not in bufs:
        bufs["x"] = torch.empty((n_r, n_c, n_c, k), dtype=torch.float32, device=y.device)
    vb, ve = vox if vox is not None else (0, 0)
    bb, be = bins if bins is not None else (0, n_k)
    if vox is not None and "xh" not in bufs:
        bufs["xh"] = torch.empty((ve - vb, be - bb), dtype=torch.float32, device=y.device)
    xh = bufs.get("xh") if vox is not None else None
    opts = NmfOpts(k, algo, precision, init, max_iter, check_every, polish_rounds, polish_algo, polish_bf16_rounds,
                   rel_obj_tol, f_ref, mlp.handle if mlp is not None else None, None, None,
                   float(mlp_fallback_rel), int(bool(anls_extrapolate)))
    hist = (C.c_double * max(history_cap, 1))()
    stats = NmfStats(0, 0, 0.0, 0.0, C.cast(hist, C.POINTER(C.c_double)), history_cap, 0, 0.0, 0, 0)
    keep = (C.c_double * n_v)(*[float(a) for a in angles]) if angles is not None else None
    yd = F32 if y.dtype == torch.float32 else U16
    od = F32 if yo.dtype == torch.float32 else U16
    _check(_lib.hsn_fhr_step(ctx, C.byref(dims), _ptr(y), yd, _ptr(yo), od, float(count_floor), _ptr(bufs["p"]), ldp,
                             _ptr(pb), ldb if pb is not None else 0, _ptr(bufs.get("pooled") if learned else None),
                             _ptr(V), _ptr(D), C.byref(opts), C.byref(stats), keep, int(cgls_iters), _ptr(bufs["x"]),
                             vb, ve, bb, be, _ptr(xh), be - bb, _stream(dev)), ctx)
    return bufs["x"], xh, _stats(stats, hist)


def hsn_mbir(sino: torch.Tensor, sigma_v, sigma_x, p: float = 1.2, T: float = 1.0, n_outer: int = 10,
             n_inner: int = 5, x0: Optional[torch.Tensor] = None, angles: Optional[Sequence[float]] = None):
    """qGGMRF-MBIR per channel: sino [N_v][N_r][N][K] -> x [N_r][N][N][K].  sigma_v, sigma_x: a
    scalar or K values; x0: the start (default zeros), copied."""
    _need(sino, "sino", torch.float32, shape=(None, None, None, None))
    n_v, n_r, n, k = sino.shape
    _opt(x0, "x0", (torch.float32, torch.float64), shape=(n_r, n, n, k), layout=None, device=sino.device)
    dev = _dev(sino)
    ctx = context(dev)
    g, keep = _geom(n_v, n_r, n, k, angles)

    def per_channel(v):
        vals = [float(t) for t in v] if hasattr(v, "__len__") else [float(v)] * k
        if len(vals) != k:
            raise ValueError(f"expected {k} per-channel values, got {len(vals)}")
        return (C.c_double * k)(*vals)

    sv, sx = per_channel(sigma_v), per_channel(sigma_x)
    if x0 is None:
        x = torch.zeros((n_r, n, n, k), dtype=torch.float32, device=sino.device)
    else:
        x = x0.to(device=sino.device, dtype=torch.float32).contiguous().clone()
    _check(_lib.hsn_mbir(ctx, C.byref(g), _ptr(sino), _ptr(x), sv, sx, float(p), float(T), int(n_outer),
                         int(n_inner), _stream(dev)), ctx)
    return x


def hsn_fbp(sino: torch.Tensor, n_views: int, n_slices: int, n: int, k: int,
            angles: Optional[Sequence[float]] = None, ld: Optional[int] = None,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Filtered backprojection of k-channel rays (ray i at sino.data_ptr() + i * ld floats;
    ld = k: sino is [N_v][N_r][N][k]) -> x [N_r][N][N][k]."""
    ld_ = int(ld or k)
    _need(sino, "sino", torch.float32, layout="inner", extent=(n_views * n_slices * n - 1) * ld_ + k)
    _opt(out, "out", torch.float32, shape=(n_slices, n, n, k), device=sino.device)
    dev = _dev(sino)
    ctx = context(dev)
    g, keep = _geom(n_views, n_slices, n, k, angles)
    if out is None:
        out = torch.empty((n_slices, n, n, k), dtype=torch.float32, device=sino.device)
    _check(_lib.hsn_fbp(ctx, C.byref(g), _ptr(sino), int(ld or k), _ptr(out), _stream(dev)), ctx)
    return out


def hsn_rehydrate(xs: torch.Tensor, D: torch.Tensor, vox=None, bins=None) -> torch.Tensor:
    """x^h = x^s D^T over [vox[0], vox[1]) x [bins[0], bins[1])."""
    _need(xs, "xs", torch.float32, shape=(None, None))
    _need(D, "D", torch.float32, shape=(None, xs.shape[1]), device=xs.device)
    dev = _dev(xs)
    ctx = context(dev)
    n_x, k = xs.shape
    n_k = D.shape[0]
    vb, ve = vox if vox is not None else (0, n_x)
    bb, be = bins if bins is not None else (0, n_k)
    out = torch.empty((ve - vb, be - bb), dtype=torch.float32, device=xs.device)
    _check(_lib.hsn_rehydrate(ctx, _ptr(xs), _ptr(D), n_x, n_k, k, vb, ve, bb, be, _ptr(out), be - bb,
                              _stream(dev)), ctx)
    return out


def bf16_bits_to_float(t: torch.Tensor) -> torch.Tensor:
    """View int16 bfloat16 bits as float32 (for checks)."""
    return (t.to(torch.int32) << 16).view(torch.float32) if t.dtype == torch.int16 else t


def hsn_profile_enable(on: bool = True, device: int = 0) -> None:
    ctx = context(device)
    _check(_lib.hsn_profile_enable(ctx, int(on)), ctx)


def hsn_profile_read(kernel: int, reset: bool = True, device: int = 0):
    """(summed device ms, launches) of one kernel kind since the last reset."""
    ctx = context(device)
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(_lib.hsn_profile_read(ctx, kernel, C.byref(ms), C.byref(n), int(reset)), ctx)
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Learned warm start
# ---------------------------------------------------------------------------

def hsn_mlp_n_params(k: int) -> int:
    return int(_lib.hsn_mlp_n_params(k))


class Mlp:
    """Owner of an hsn_mlp handle (256-128-128-K network on one device)."""

    def __init__(self, handle, device: int):
        self.handle = handle
        self.device = device
        self.k = int(_lib.hsn_mlp_k(handle))
        self.precision = int(_lib.hsn_mlp_precision(handle))
        self.n_params = hsn_mlp_n_params(self.k)

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hsn_mlp_destroy(self.handle)
            self.handle = None

    @property
    def x_dtype(self):
        return torch.int16 if self.precision == PREC_BF16 else torch.float32

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, np.float32)
        ctx = context(self.device)
        _check(_lib.hsn_mlp_get_params(ctx, self.handle, _P(out.ctypes.data)), ctx)
        return out

    def set_params(self, params) -> None:
        import numpy as np
        a = np.ascontiguousarray(params, np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        ctx = context(self.device)
        _check(_lib.hsn_mlp_set_params(ctx, self.handle, _P(a.ctypes.data)), ctx)


def hsn_mlp_create(k: int, precision: int = PREC_BF16, params=None, device: int = 0) -> Mlp:
    import numpy as np
    ctx = context(device)
    h = _P()
    a = None if params is None else np.ascontiguousarray(params, np.float32)
    if a is not None and a.size != hsn_mlp_n_params(k):
        raise ValueError("wrong parameter count")
    _check(_lib.hsn_mlp_create(ctx, C.byref(h), k, precision, None if a is None else _P(a.ctypes.data)), ctx)
    return Mlp(h, device)


def hsn_mlp_pool(p_bf16: torch.Tensor, n_k: int, x_dtype: int = PREC_BF16) -> torch.Tensor:
    """[N_p][ldb] bfloat16 bits -> [N_p][256] pooled (int16 bits or float32)."""
    _need(p_bf16, "p_bf16", _U16, shape=(None, None), layout="rows")
    if p_bf16.shape[1] < n_k:
        raise ValueError(f"hsn: p_bf16 rows must hold n_k = {n_k} bins")
    dev = _dev(p_bf16)
    ctx = context(dev)
    n_p = p_bf16.shape[0]
    x = torch.empty((n_p, MLP_IN), dtype=torch.int16 if x_dtype == PREC_BF16 else torch.float32,
                    device=p_bf16.device)
    _check(_lib.hsn_mlp_pool(ctx, _ptr(p_bf16), p_bf16.stride(0), n_p, n_k, x_dtype, _ptr(x), _stream(dev)), ctx)
    return x


def hsn_mlp_forward(mlp: Mlp, x: torch.Tensor) -> torch.Tensor:
    _need(x, "x", mlp.x_dtype, shape=(None, MLP_IN))
    dev = _dev(x)
    ctx = context(dev)
    y = torch.empty((x.shape[0], mlp.k), dtype=torch.float32, device=x.device)
    _check(_lib.hsn_mlp_forward(ctx, mlp.handle, _ptr(x), x.shape[0], _ptr(y), _stream(dev)), ctx)
    return y


def hsn_mlp_loss_grad(mlp: Mlp, x: torch.Tensor, target: torch.Tensor):
    """(mean squared error, flat gradient [n_params]) over all rows as one batch."""
    _need(x, "x", mlp.x_dtype, shape=(None, MLP_IN))
    _need(target, "target", torch.float32, shape=(x.shape[0], mlp.k), device=x.device)
    dev = _dev(x)
    ctx = context(dev)
    g = torch.empty(mlp.n_params, dtype=torch.float32, device=x.device)
    loss = torch.empty((), dtype=torch.float64, device=x.device)
    _check(_lib.hsn_mlp_loss_grad(ctx, mlp.handle, _ptr(x), _ptr(target), x.shape[0], _ptr(g), _ptr(loss),
                                  _stream(dev)), ctx)
    return loss, g


def hsn_mlp_train(mlp: Mlp, x: torch.Tensor, target: torch.Tensor, epochs: int, batch: int = 4096,
                  lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, seed: int = 0):
    """Adam over shuffled mini-batches; returns the per-epoch mean batch loss."""
    _need(x, "x", mlp.x_dtype, shape=(None, MLP_IN))
    _need(target, "target", torch.float32, shape=(x.shape[0], mlp.k), device=x.device)
    dev = _dev(x)
    ctx = context(dev)
    o = TrainOpts(epochs, batch, lr, beta1, beta2, eps, seed)
    hist = (C.c_double * max(epochs, 1))()
    _check(_lib.hsn_mlp_train(ctx, mlp.handle, _ptr(x), _ptr(target), x.shape[0], C.byref(o),
                              C.cast(hist, _P), _stream(dev)), ctx)
    return [hist[i] for i in range(epochs)]


def hsn_mlp_infer(mlp: Mlp, p_bf16: torch.Tensor, n_k: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _need(p_bf16, "p_bf16", _U16, shape=(None, None), layout="rows")
    if p_bf16.shape[1] < n_k:
        raise ValueError(f"hsn: p_bf16 rows must hold n_k = {n_k} bins")
    _opt(out, "out", torch.float32, shape=(p_bf16.shape[0], mlp.k), device=p_bf16.device)
    dev = _dev(p_bf16)
    ctx = context(dev)
    n_p = p_bf16.shape[0]
    if out is None:
        out = torch.empty((n_p, mlp.k), dtype=torch.float32, device=p_bf16.device)
    _check(_lib.hsn_mlp_infer(ctx, mlp.handle, _ptr(p_bf16), p_bf16.stride(0), n_p, n_k, _ptr(out),
                              _stream(dev)), ctx)
    return out


def hsn_mlp_save(mlp: Mlp, path: str) -> None:
    ctx = context(mlp.device)
    _check(_lib.hsn_mlp_save(ctx, mlp.handle, os.fsencode(path)), ctx)


def hsn_mlp_load(path: str, device: int = 0) -> Mlp:
    ctx = context(device)
    h = _P()
    _check(_lib.hsn_mlp_load(ctx, C.byref(h), os.fsencode(path)), ctx)
    return Mlp(h, device)


def hsn_canonicalize(V: torch.Tensor, D: torch.Tensor, library: Optional[torch.Tensor] = None) -> None:
    """In place: unit-norm D columns, V scaled inversely, columns matched to library (or by |V|)."""
    _need(V, "V", torch.float32, shape=(None, None))
    _need(D, "D", torch.float32, shape=(None, V.shape[1]), device=V.device)
    _opt(library, "library", torch.float32, shape=tuple(D.shape), device=V.device)
    dev = _dev(V)
    ctx = context(dev)
    n_p, k = V.shape
    _check(_lib.hsn_canonicalize(ctx, _ptr(V), n_p, _ptr(D), D.shape[0], k, _ptr(library), _stream(dev)), ctx)


def hsn_fmd(xs: torch.Tensor, labels: torch.Tensor, n_m: int, Ds: torch.Tensor):
    """Alg. 2 tail: (T [n_m][K], x^m [n_x][n_m], D^m [n_k][n_m]) from x^s [n_x][K],
    int32 labels [n_x] (-1 = no region) and D^s [n_k][K]."""
    _need(xs, "xs", torch.float32, shape=(None, None))
    _need(labels, "labels", torch.int32, shape=(xs.shape[0],), device=xs.device)
    _need(Ds, "Ds", torch.float32, shape=(None, xs.shape[1]), device=xs.device)
    dev = _dev(xs)
    ctx = context(dev)
    n_x, k = xs.shape
    n_k = Ds.shape[0]
    T = torch.empty((n_m, k), dtype=torch.float32, device=xs.device)
    xm = torch.empty((n_x, n_m), dtype=torch.float32, device=xs.device)
    Dm = torch.empty((n_k, n_m), dtype=torch.float32, device=xs.device)
    _check(_lib.hsn_fmd(ctx, _ptr(xs), n_x, k, _ptr(labels), n_m, _ptr(Ds), n_k, _ptr(T), _ptr(xm), _ptr(Dm),
                        _stream(dev)), ctx)
    return T, xm, Dm
