"""MI355X (gfx950) tile rasterizer hot path of progressive 3D Gaussian Splatting.

Thin Python binding over the C ABI in include/gs.h (libgsmi.so, built in-tree by
_build.py).  Every function has the name of the C entry point it calls and only
marshals arguments: device pointers are taken from integers or from objects with
a ``data_ptr()`` method (torch tensors), streams from integers or from the current
torch stream, cameras from dicts with R, t, fx, fy, cx, cy, width, height, bg.
All work runs in the library's HIP kernels; there is no fallback path: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmi.so")

GS_OK, GS_ERR_INVALID, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED, GS_ERR_STATE = 0, -1, -2, -3, -4, -5
GS_MAX_VIEWS = 64
(GS_GROUP_MEAN, GS_GROUP_SCALE, GS_GROUP_ROT, GS_GROUP_OPACITY, GS_GROUP_SH_DC, GS_GROUP_SH_REST) = range(6)
GS_N_GROUPS = 6
(GS_BUF_RECORDS, GS_BUF_DEPTH, GS_BUF_TOUCHED, GS_BUF_TILE_RECT, GS_BUF_KEYS, GS_BUF_VALUES, GS_BUF_RANGES,
 GS_BUF_T_FINAL, GS_BUF_N_CONTRIB, GS_BUF_LAST, GS_BUF_GRAD2D, GS_BUF_PAIR_VIEW, GS_BUF_ALPHA_SUM,
 GS_BUF_EVALS, GS_BUF_PAIRS_EFF) = range(15)
(GS_K_PREPROCESS, GS_K_DEPTH_SORT, GS_K_SCAN, GS_K_EMIT, GS_K_TILE_SORT, GS_K_RANGES, GS_K_RENDER_FWD, GS_K_LOSS,
 GS_K_RENDER_BWD, GS_K_PREPROCESS_BWD, GS_K_ADAM, GS_K_ZERO, GS_K_LOAD, GS_K_BWD_ADAM) = range(14)
KERNEL_NAMES = ["preprocess", "depth_sort", "scan", "emit", "tile_sort", "ranges", "render_fwd", "loss",
                "render_bwd", "preprocess_bwd", "adam", "zero", "load", "preprocess_bwd_adam"]

_STATUS = {0: "GS_OK", -1: "GS_ERR_INVALID", -2: "GS_ERR_CAPACITY", -3: "GS_ERR_HIP", -4: "GS_ERR_UNSUPPORTED",
           -5: "GS_ERR_STATE"}

# Exported symbols (must match include/gs.h).
EXPORTS = ["gs_abi_version", "gs_create", "gs_destroy", "gs_last_error", "gs_layout", "gs_preprocess", "gs_bin_sort",
           "gs_render_fwd", "gs_loss", "gs_loss_noalloc", "gs_load_balance", "gs_render_bwd", "gs_adam_step", "gs_render_bwd_adam",
           "gs_set_cull", "gs_set_backward_order", "gs_buffer_size", "gs_sync_status", "gs_reserve_pairs",
           "gs_copy_buffer", "gs_profile_enable", "gs_profile_read", "gs_memory_bytes", "gs_render_count",
           "gs_probe_copy", "gs_probe_fma", "gs_sched_weights",
           "gs_sched_plan", "gs_sched_lr"]
GS_CULL_RECT, GS_CULL_ELLIPSE, GS_CULL_ELLIPSE_EXACT = 0, 1, 2
GS_BWD_ATOMIC, GS_BWD_ORDERED = 0, 1


class GsError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {message}")
        self.status = status


class GsCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("bg", ctypes.c_float * 3)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_D = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)
_LP = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python paper_2503_13086_amd/_build.py")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "gs_abi_version": (_I32, []),
        "gs_create": (_I32, [ctypes.POINTER(_P), _I32]),
        "gs_destroy": (None, [_P]),
        "gs_last_error": (ctypes.c_char_p, [_P]),
        "gs_layout": (_I32, [ctypes.POINTER(GsCamera), _I32, _I32, ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64)]),
        "gs_preprocess": (_I32, [_P, _P, _I32, _I32, _I32, ctypes.POINTER(GsCamera), _I32, _I32, _P]),
        "gs_bin_sort": (_I32, [_P, ctypes.POINTER(ctypes.c_int64), _P]),
        "gs_sync_status": (_I32, [_P, _P]),
        "gs_reserve_pairs": (_I32, [_P, ctypes.c_int64, _P]),
        "gs_render_fwd": (_I32, [_P, _P, _P]),
        "gs_loss": (_I32, [_P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
        "gs_loss_noalloc": (_I32, [_P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
        "gs_render_bwd": (_I32, [_P, _P, _P, _P, _I32, _P]),
        "gs_load_balance": (_I32, [_P, ctypes.c_float, _P, _P]),
        "gs_adam_step": (_I32, [_P, _P, _P, _P, _P, _P, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), _I32, ctypes.c_uint32, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, _P]),
        "gs_render_bwd_adam": (_I32, [_P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float), _I32, ctypes.c_uint32, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, _P]),
        "gs_set_cull": (_I32, [_P, _I32]),
        "gs_set_backward_order": (_I32, [_P, _I32]),
        "gs_buffer_size": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_size_t)]),
        "gs_copy_buffer": (_I32, [_P, _I32, _P, ctypes.c_size_t, _P]),
        "gs_profile_enable": (_I32, [_P, _I32]),
        "gs_profile_read": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
        "gs_memory_bytes": (_I32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
        "gs_render_count": (_I32, [_P, _P]),
        "gs_probe_copy": (_I32, [_P, _P, ctypes.c_size_t, _P]),
        "gs_probe_fma": (_I32, [_P, _I32, _I32, ctypes.POINTER(ctypes.c_int64), _P]),
        "gs_sched_weights": (_I32, [_D, _I32, _I32, _D, _IP]),
        "gs_sched_plan": (_I32, [_D, _I32, _I32, _I32, _D, _IP, _IP]),
        "gs_sched_lr": (_I32, [_LP, _D, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def lib():
    return _load()


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def _check(ctx, st: int, where: str):
    if st != GS_OK:
        msg = _load().gs_last_error(ctx).decode() if ctx else ""
        raise GsError(st, where, msg)


def cameras(cams: Sequence[dict]):
    """ctypes array of GsCamera from camera dicts."""
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        R = [float(x) for x in list(getattr(c["R"], "ravel", lambda: c["R"])())]
        arr[i].R[:] = R
        arr[i].t[:] = [float(x) for x in c["t"]]
        arr[i].fx, arr[i].fy = float(c["fx"]), float(c["fy"])
        arr[i].cx, arr[i].cy = float(c["cx"]), float(c["cy"])
        arr[i].width, arr[i].height = int(c["width"]), int(c["height"])
        arr[i].bg[:] = [float(x) for x in c.get("bg", (0.0, 0.0, 0.0))]
    return arr


def gs_abi_version() -> int:
    return _load().gs_abi_version()


def gs_create(device: int = 0):
    h = _P()
    st = _load().gs_create(ctypes.byref(h), device)
    if st != GS_OK:
        raise GsError(st, "gs_create", f"device {device} unavailable")
    return h.value


def gs_destroy(ctx) -> None:
    _load().gs_destroy(ctx)


def gs_last_error(ctx) -> str:
    return _load().gs_last_error(ctx).decode()


def gs_layout(cams: Sequence[dict], tile: int = 16):
    arr = cameras(cams)
    n = len(cams)
    po = (ctypes.c_int64 * (n + 1))()
    to = (ctypes.c_int64 * (n + 1))()
    _check(None, _load().gs_layout(arr, n, tile, po, to), "gs_layout")
    return list(po), list(to)


def gs_preprocess(ctx, params, n: int, stride: int, sh_degree: int, cams: Sequence[dict], tile: int = 16,
                  stream=None) -> None:
    arr = cameras(cams)
    _check(ctx, _load().gs_preprocess(ctx, _ptr(params), n, stride, sh_degree, arr, len(cams), tile,
                                      _stream(stream)), "gs_preprocess")


def gs_bin_sort(ctx, stream=None, count: bool = True) -> Optional[int]:
    """Returns K when count is True (the call then waits for the device); with
    count False K stays on the device and None is returned."""
    if not count:
        _check(ctx, _load().gs_bin_sort(ctx, None, _stream(stream)), "gs_bin_sort")
        return None
    k = ctypes.c_int64(0)
    _check(ctx, _load().gs_bin_sort(ctx, ctypes.byref(k), _stream(stream)), "gs_bin_sort")
    return k.value


def gs_sync_status(ctx, stream=None) -> None:
    """Raises GsError (GS_ERR_CAPACITY) when the last binning ran out of room."""
    _check(ctx, _load().gs_sync_status(ctx, _stream(stream)), "gs_sync_status")


def gs_reserve_pairs(ctx, n_pairs: int, stream=None) -> None:
    _check(ctx, _load().gs_reserve_pairs(ctx, int(n_pairs), _stream(stream)), "gs_reserve_pairs")


def gs_render_fwd(ctx, color, stream=None) -> None:
    _check(ctx, _load().gs_render_fwd(ctx, _ptr(color), _stream(stream)), "gs_render_fwd")


def gs_loss(ctx, color, target, w_l1: float, w_dssim: float, loss_out, dL_dcolor, stream=None) -> None:
    _check(ctx, _load().gs_loss(ctx, _ptr(color), _ptr(target), w_l1, w_dssim, _ptr(loss_out), _ptr(dL_dcolor),
                                _stream(stream)), "gs_loss")


def gs_loss_noalloc(ctx, color, target, w_l1: float, w_dssim: float, loss_out, dL_dcolor, stream=None) -> None:
    _check(ctx, _load().gs_loss_noalloc(ctx, _ptr(color), _ptr(target), w_l1, w_dssim, _ptr(loss_out),
                                        _ptr(dL_dcolor), _stream(stream)), "gs_loss_noalloc")


def gs_load_balance(ctx, w_load: float, loss_out=None, stream=None) -> None:
    _check(ctx, _load().gs_load_balance(ctx, w_load, _ptr(loss_out), _stream(stream)), "gs_load_balance")


def gs_render_bwd(ctx, params, dL_dcolor, grad, accumulate: bool = False, stream=None) -> None:
    _check(ctx, _load().gs_render_bwd(ctx, _ptr(params), _ptr(dL_dcolor), _ptr(grad), 1 if accumulate else 0,
                                      _stream(stream)), "gs_render_bwd")


def gs_adam_step(ctx, params, grad, m, v, step, n: int, stride: int, sh_degree: int, lr_group: Sequence[float],
                 view_lr_scale: Optional[Sequence[float]] = None, group_mask: int = 1, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-15, stream=None) -> None:
    lg = (ctypes.c_float * GS_N_GROUPS)(*[float(x) for x in lr_group])
    if view_lr_scale is not None and len(view_lr_scale) > 0:
        vs = (ctypes.c_float * len(view_lr_scale))(*[float(x) for x in view_lr_scale])
        nv = len(view_lr_scale)
    else:
        vs, nv = None, 0
    _check(ctx, _load().gs_adam_step(ctx, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), n, stride,
                                     sh_degree, lg, vs, nv, group_mask, beta1, beta2, eps, _stream(stream)),
           "gs_adam_step")


def gs_render_bwd_adam(ctx, params, dL_dcolor, grad, m, v, step, lr_group: Sequence[float],
                       view_lr_scale: Optional[Sequence[float]] = None, group_mask: int = 1, beta1: float = 0.9,
                       beta2: float = 0.999, eps: float = 1e-15, stream=None) -> None:
    """gs_render_bwd (overwrite) + gs_adam_step in one pass; grad may be None."""
    lg = (ctypes.c_float * GS_N_GROUPS)(*[float(x) for x in lr_group])
    if view_lr_scale is not None and len(view_lr_scale) > 0:
        vs = (ctypes.c_float * len(view_lr_scale))(*[float(x) for x in view_lr_scale])
        nv = len(view_lr_scale)
    else:
        vs, nv = None, 0
    _check(ctx, _load().gs_render_bwd_adam(ctx, _ptr(params), _ptr(dL_dcolor), _ptr(grad), _ptr(m), _ptr(v),
                                           _ptr(step), lg, vs, nv, group_mask, beta1, beta2, eps, _stream(stream)),
           "gs_render_bwd_adam")


def gs_set_cull(ctx, mode: int) -> None:
    _check(ctx, _load().gs_set_cull(ctx, mode), "gs_set_cull")


def gs_set_backward_order(ctx, mode: int) -> None:
    _check(ctx, _load().gs_set_backward_order(ctx, mode), "gs_set_backward_order")


def gs_buffer_size(ctx, which: int) -> int:
    b = ctypes.c_size_t(0)
    _check(ctx, _load().gs_buffer_size(ctx, which, ctypes.byref(b)), "gs_buffer_size")
    return b.value


def gs_copy_buffer(ctx, which: int, dst, nbytes: int, stream=None) -> None:
    _check(ctx, _load().gs_copy_buffer(ctx, which, _ptr(dst), nbytes, _stream(stream)), "gs_copy_buffer")


def gs_profile_enable(ctx, enable: bool = True) -> None:
    _check(ctx, _load().gs_profile_enable(ctx, 1 if enable else 0), "gs_profile_enable")


def gs_profile_read(ctx, kernel: int):
    n = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    _check(ctx, _load().gs_profile_read(ctx, kernel, ctypes.byref(n), ctypes.byref(t)), "gs_profile_read")
    return n.value, t.value


def gs_memory_bytes(ctx) -> int:
    b = ctypes.c_size_t(0)
    _check(ctx, _load().gs_memory_bytes(ctx, ctypes.byref(b)), "gs_memory_bytes")
    return b.value


def gs_render_count(ctx, stream=None) -> None:
    """Per-pixel count of the Gaussians evaluated up to termination (GS_BUF_EVALS)."""
    _check(ctx, _load().gs_render_count(ctx, _stream(stream)), "gs_render_count")


def gs_probe_copy(src, dst, nbytes: int, stream=None) -> None:
    """Streaming copy probe of nbytes (multiple of 16) from src to dst (device tensors)."""
    _check(None, _load().gs_probe_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "gs_probe_copy")


def gs_probe_fma(out, blocks: int, iters: int, stream=None) -> int:
    """fp32 FMA-rate probe writing blocks x 256 floats to out; returns its flop count."""
    f = ctypes.c_int64(0)
    _check(None, _load().gs_probe_fma(_ptr(out), int(blocks), int(iters), ctypes.byref(f), _stream(stream)),
           "gs_probe_fma")
    return f.value


def _f64_array(x, n=None):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(_D)


def gs_sched_weights(overlap, new_image: int):
    """Eq. 3-4 weights (-1 = unreached) and layers of every image; host only."""
    import numpy as np
    M, pM = _f64_array(overlap)
    n = int(round(M.size ** 0.5))
    if M.shape != (n, n):
        raise ValueError("overlap must be a square matrix")
    w = np.empty(n, np.float64)
    lay = np.empty(n, np.int32)
    _check(None, _load().gs_sched_weights(pM, n, new_image, w.ctypes.data_as(_D), lay.ctypes.data_as(_IP)),
           "gs_sched_weights")
    return w, lay


def gs_sched_plan(weights, n_m: int, t_i: int, u):
    """Image trained by each of the t_i iterations of an arrival, and the Eq. 5
    local shares; host only."""
    import numpy as np
    w, pw = _f64_array(weights)
    n = w.size
    uu, pu = _f64_array(u, n)
    plan = np.empty(max(t_i, 1), np.int32)
    share = np.empty(n, np.int32)
    _check(None, _load().gs_sched_plan(pw, n, n_m, t_i, pu, plan.ctypes.data_as(_IP), share.ctypes.data_as(_IP)),
           "gs_sched_plan")
    return plan[:t_i], share


def gs_sched_lr(trained, overlap, eta0: float, etaf: float, t_a: float):
    """Eq. 6-7 current rates and Eq. 8 rates of every image; host only."""
    import numpy as np
    T = np.ascontiguousarray(np.asarray(trained, dtype=np.int64))
    n = T.size
    M, pM = _f64_array(overlap, n * n)
    cur = np.empty(n, np.float64)
    lr = np.empty(n, np.float64)
    _check(None, _load().gs_sched_lr(T.ctypes.data_as(_LP), pM, n, eta0, etaf, t_a, cur.ctypes.data_as(_D),
                                     lr.ctypes.data_as(_D)), "gs_sched_lr")
    return cur, lr
