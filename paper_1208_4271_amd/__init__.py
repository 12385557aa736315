"""Python binding of the micx C ABI (include/micx.h): MINE statistics on MI355X.

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``libmicx.so``; PyTorch supplies device memory and streams.  There
is no CPU fallback: importing works without the library, but every call
raises if ``libmicx.so`` has not been built (``python -m
paper_1208_4271_amd._build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmicx.so")

MICX_OK = 0
MICX_EINVAL = -1
MICX_ESMALLN = -2
MICX_ENONFINITE = -3
MICX_ENOMEM = -4
MICX_EDEVICE = -5
MICX_ETOOBIG = -6
MAX_N = 8192

F32, F64, I32 = 0, 1, 2
MODE_FP64 = 0
MODE_DP32 = 1

# Compatibility variants (include/micx.h, MICX_COMPAT_*); same bit values as
# the oracle's reading flags.
COMPAT_TIE_STRICT = 1
COMPAT_DESIRED_INT = 2
COMPAT_COMBINE_INDEX = 4
COMPAT_NORM_BY_Y = 8
COMPAT_BOUND_STRICT = 16
COMPAT_KHAT_PLUS1 = 32

# Every symbol declared in include/micx.h.
EXPORTS = (
    "micx_ctx_create", "micx_ctx_destroy", "micx_check_param", "micx_grid_bound",
    "micx_compute_score", "micx_mic", "micx_mas", "micx_mev", "micx_mcn", "micx_free_score",
    "micx_allpairs", "micx_pairs", "micx_batch", "micx_debug_item", "micx_strerror",
    "micx_set_profiling", "micx_get_profile", "micx_set_dp32_tolerance", "micx_set_compat",
    "micx_pearson", "micx_score_noalloc", "micx_status", "micx_set_graphs", "micx_debug_tables",
    "micx_autotune", "micx_tune_save", "micx_tune_load", "micx_tune_clear", "micx_dp32_bound",
)

# Size of the device array behind micx_score_noalloc (include/micx.h).
NOALLOC_BYTES = 32 << 20


class MicxError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s: %s (code %d)" % (where, strerror(code), code))


class _Score(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("B", ctypes.c_int), ("W", ctypes.c_int),
                ("M", ctypes.POINTER(ctypes.c_double)), ("Axy", ctypes.POINTER(ctypes.c_double)),
                ("Ayx", ctypes.POINTER(ctypes.c_double)), ("stats", ctypes.c_double * 4)]


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("x", ctypes.POINTER(ctypes.c_double)),
                ("y", ctypes.POINTER(ctypes.c_double))]


class _Param(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("c", ctypes.c_double)]


def _param(alpha, c):
    return _Param(float(alpha), float(c))


class _PairDesc(ctypes.Structure):
    _fields_ = [("off_x", ctypes.c_int64), ("off_y", ctypes.c_int64), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("alpha", ctypes.c_double), ("c", ctypes.c_double)]


class _Profile(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int64), ("dp_cells", ctypes.c_int64),
                ("h_evals", ctypes.c_int64), ("h_terms", ctypes.c_int64),
                ("dp_ms", ctypes.c_double), ("dp_launches", ctypes.c_int),
                ("dp32_classes", ctypes.c_int), ("fp64_classes", ctypes.c_int),
                ("dp32_bound", ctypes.c_double), ("recheck_pairs", ctypes.c_int64),
                ("recheck_items", ctypes.c_int64), ("recheck_ms", ctypes.c_double),
                ("coop_classes", ctypes.c_int), ("host_ms", ctypes.c_double)]


_lib = None
_ctxs = {}


def load_library():
    """Load libmicx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmicx.so is not built: run `python -m paper_1208_4271_amd._build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp, ip, vp = P(ctypes.c_double), P(ctypes.c_int), ctypes.c_void_p
    lib.micx_ctx_create.argtypes = [P(vp), ctypes.c_int]
    lib.micx_ctx_create.restype = ctypes.c_int
    lib.micx_ctx_destroy.argtypes = [vp]
    lib.micx_ctx_destroy.restype = None
    lib.micx_check_param.argtypes = [P(_Param)]
    lib.micx_check_param.restype = ctypes.c_char_p
    lib.micx_grid_bound.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.micx_grid_bound.restype = ctypes.c_int
    lib.micx_compute_score.argtypes = [vp, P(_Problem), P(_Param), ctypes.c_int, P(P(_Score))]
    lib.micx_compute_score.restype = ctypes.c_int
    for f in ("micx_mic", "micx_mas", "micx_mev"):
        getattr(lib, f).argtypes = [P(_Score)]
        getattr(lib, f).restype = ctypes.c_double
    lib.micx_mcn.argtypes = [P(_Score), ctypes.c_double]
    lib.micx_mcn.restype = ctypes.c_double
    lib.micx_free_score.argtypes = [P(_Score)]
    lib.micx_free_score.restype = None
    lib.micx_allpairs.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(_Param),
                                  ctypes.c_int, vp, vp]
    lib.micx_allpairs.restype = ctypes.c_int
    lib.micx_autotune.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(_Param),
                                  ctypes.c_int, ctypes.c_char_p, vp]
    lib.micx_autotune.restype = ctypes.c_int
    for f in ("micx_tune_save", "micx_tune_load"):
        getattr(lib, f).argtypes = [ctypes.c_char_p]
        getattr(lib, f).restype = ctypes.c_int
    lib.micx_tune_clear.argtypes = []
    lib.micx_tune_clear.restype = ctypes.c_int
    lib.micx_status.argtypes = [vp]
    lib.micx_status.restype = ctypes.c_int
    lib.micx_set_graphs.argtypes = [vp, ctypes.c_int]
    lib.micx_set_graphs.restype = ctypes.c_int
    lib.micx_pairs.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_int32),
                               ctypes.c_int64, P(_Param), ctypes.c_int, vp, vp]
    lib.micx_pairs.restype = ctypes.c_int
    lib.micx_batch.argtypes = [vp, vp, ctypes.c_int, P(_PairDesc), ctypes.c_int64, ctypes.c_int, vp, vp]
    lib.micx_batch.restype = ctypes.c_int
    lib.micx_pearson.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_int32),
                                 ctypes.c_int64, vp, vp, vp]
    lib.micx_pearson.restype = ctypes.c_int
    lib.micx_score_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, P(_Param),
                                       ctypes.c_int, vp, vp, vp, vp]
    lib.micx_score_noalloc.restype = ctypes.c_int
    lib.micx_debug_item.argtypes = [vp, P(_Problem), P(_Param), ctypes.c_int, ctypes.c_int,
                                    ip, ip, ip, ip, ip]
    lib.micx_debug_item.restype = ctypes.c_int
    lib.micx_debug_tables.argtypes = [vp, P(_Problem), P(_Param), ctypes.c_int, ctypes.c_int, ip, ip, ip]
    lib.micx_debug_tables.restype = ctypes.c_int
    lib.micx_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.micx_set_profiling.restype = ctypes.c_int
    lib.micx_get_profile.argtypes = [vp, P(_Profile)]
    lib.micx_get_profile.restype = ctypes.c_int
    lib.micx_set_dp32_tolerance.argtypes = [vp, ctypes.c_double]
    lib.micx_set_dp32_tolerance.restype = ctypes.c_int
    lib.micx_dp32_bound.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.micx_dp32_bound.restype = ctypes.c_double
    lib.micx_set_compat.argtypes = [vp, ctypes.c_int]
    lib.micx_set_compat.restype = ctypes.c_int
    lib.micx_strerror.argtypes = [ctypes.c_int]
    lib.micx_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().micx_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != MICX_OK:
        raise MicxError(rc, where)


def context(device: int = 0):
    """The library context of a device (created once per process)."""
    if device not in _ctxs:
        h = ctypes.c_void_p()
        _check(load_library().micx_ctx_create(ctypes.byref(h), int(device)), "micx_ctx_create")
        _ctxs[device] = h
    return _ctxs[device]


def check_param(alpha: float, c: float):
    p = _param(alpha, c)
    msg = load_library().micx_check_param(ctypes.byref(p))
    return None if msg is None else msg.decode()


def status(device: int = 0) -> int:
    """micx_status: waits for the last pair call's work and returns its
    device-side result code."""
    return load_library().micx_status(context(device))


def autotune(X, alpha: float = 0.6, c: float = 15.0, mode: int = MODE_DP32, cache_path=None,
             stream=None):
    """micx_autotune: time the DP launch shapes of every row count on all pairs
    of the first min(m, 192) rows of the CUDA tensor X and keep the fastest
    (process-wide).  cache_path: file for the table, or None."""
    if not X.is_cuda or X.dim() != 2:
        raise ValueError("X must be a 2-D CUDA tensor")
    X = X.contiguous()
    dt = _DTYPES.get(str(X.dtype))
    if dt is None:
        raise ValueError("X dtype must be float32, float64 or int32")
    m, n = X.shape
    par = _param(alpha, c)
    rc = load_library().micx_autotune(context(X.device.index or 0), ctypes.c_void_p(X.data_ptr()), dt, m, n,
                                      ctypes.byref(par), int(mode),
                                      cache_path.encode() if cache_path else None, _stream_ptr(stream))
    _check(rc, "micx_autotune")


def tune_save(path):
    _check(load_library().micx_tune_save(path.encode()), "micx_tune_save")


def tune_load(path):
    _check(load_library().micx_tune_load(path.encode()), "micx_tune_load")


def tune_clear():
    _check(load_library().micx_tune_clear(), "micx_tune_clear")


def set_graphs(enable: bool = True, device: int = 0):
    """Launch graphs for allpairs (captured on the second identical call)."""
    _check(load_library().micx_set_graphs(context(device), 1 if enable else 0), "micx_set_graphs")


def grid_bound(n: int, alpha: float) -> int:
    return load_library().micx_grid_bound(int(n), float(alpha))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def compute_score(x, y, alpha: float = 0.6, c: float = 15.0, mode: int = MODE_FP64,
                  device: int = 0, mcn_eps=()):
    """Score of one pair (host arrays).  Returns dict: stats (MIC, MAS, MEV,
    MCN), M, Axy, Ayx (W x W, [rows-2, cols-2], NaN outside the grid bound), B,
    and mcn: {eps: micx_mcn(score, eps)} for every eps in mcn_eps."""
    lib = load_library()
    x, y = _f64(x), _f64(y)
    if len(x) != len(y):
        raise ValueError("x and y differ in length")
    out = ctypes.POINTER(_Score)()
    prob = _Problem(len(x), _dptr(x), _dptr(y))
    par = _param(alpha, c)
    _check(lib.micx_compute_score(context(device), ctypes.byref(prob), ctypes.byref(par), int(mode),
                                  ctypes.byref(out)), "micx_compute_score")
    try:
        s = out.contents
        W = s.W
        M = np.ctypeslib.as_array(s.M, shape=(W * W,)).reshape(W, W).copy()
        Axy = np.ctypeslib.as_array(s.Axy, shape=(W * W,)).reshape(W, W).copy()
        Ayx = np.ctypeslib.as_array(s.Ayx, shape=(W * W,)).reshape(W, W).copy()
        stats = np.array([lib.micx_mic(out), lib.micx_mas(out), lib.micx_mev(out),
                          lib.micx_mcn(out, 0.0)])
        mcn = {float(e): lib.micx_mcn(out, float(e)) for e in mcn_eps}
        return {"stats": stats, "M": M, "Axy": Axy, "Ayx": Ayx, "B": s.B, "W": W, "mcn": mcn}
    finally:
        lib.micx_free_score(out)


_DTYPES = {"torch.float32": F32, "torch.float64": F64, "torch.int32": I32}


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def allpairs(X, alpha: float = 0.6, c: float = 15.0, mode: int = MODE_FP64, out=None,
             stream=None, wait: bool = True):
    """All pairs of rows of a CUDA tensor X (m x n, float32/float64/int32).

    Returns a (m(m-1)/2, 4) float64 CUDA tensor of (MIC, MAS, MEV, MCN) in
    row-major upper-triangle order (0,1), (0,2), ..., (m-2, m-1).  The work
    is queued on the stream; with wait=True the call then waits for it and
    raises on a device-side error (micx_status)."""
    import torch
    if not X.is_cuda or X.dim() != 2:
        raise ValueError("X must be a 2-D CUDA tensor")
    X = X.contiguous()
    dt = _DTYPES.get(str(X.dtype))
    if dt is None:
        raise ValueError("X dtype must be float32, float64 or int32")
    m, n = X.shape
    npairs = m * (m - 1) // 2
    if out is None:
        out = torch.empty((npairs, 4), dtype=torch.float64, device=X.device)
    par = _param(alpha, c)
    dev = X.device.index or 0
    rc = load_library().micx_allpairs(context(dev), ctypes.c_void_p(X.data_ptr()), dt, m, n,
                                      ctypes.byref(par), int(mode), ctypes.c_void_p(out.data_ptr()),
                                      _stream_ptr(stream))
    _check(rc, "micx_allpairs")
    if wait:
        _check(status(dev), "micx_allpairs")
    return out


def pairs(X, pair_list, alpha: float = 0.6, c: float = 15.0, mode: int = MODE_FP64, out=None,
          stream=None, wait: bool = True):
    """Listed pairs (i, j) of rows of a CUDA tensor X.  Returns (npairs, 4)."""
    import torch
    if not X.is_cuda or X.dim() != 2:
        raise ValueError("X must be a 2-D CUDA tensor")
    X = X.contiguous()
    dt = _DTYPES.get(str(X.dtype))
    if dt is None:
        raise ValueError("X dtype must be float32, float64 or int32")
    m, n = X.shape
    pl = np.ascontiguousarray(np.asarray(pair_list, dtype=np.int32).reshape(-1, 2))
    if out is None:
        out = torch.empty((len(pl), 4), dtype=torch.float64, device=X.device)
    par = _param(alpha, c)
    dev = X.device.index or 0
    rc = load_library().micx_pairs(context(dev), ctypes.c_void_p(X.data_ptr()), dt,
                                   m, n, pl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(pl),
                                   ctypes.byref(par), int(mode),
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check(rc, "micx_pairs")
    if wait:
        _check(status(dev), "micx_pairs")
    return out


def pearson(X, pair_list=None, stats=None, out=None, stream=None):
    """Pearson's rho and the non-linearity index MIC - rho^2 (see micx_pearson)
    for the listed pairs (i, j) of rows of a CUDA tensor X, or for all pairs
    i < j in allpairs order when pair_list is None.  stats: the (npairs, 4)
    float64 CUDA output of allpairs/pairs for the same pairs, or None.
    Returns an (npairs, 2) float64 CUDA tensor of (rho, MIC - rho^2)."""
    import torch
    if not X.is_cuda or X.dim() != 2:
        raise ValueError("X must be a 2-D CUDA tensor")
    X = X.contiguous()
    dt = _DTYPES.get(str(X.dtype))
    if dt is None:
        raise ValueError("X dtype must be float32, float64 or int32")
    m, n = X.shape
    if pair_list is None:
        pl, npairs = None, m * (m - 1) // 2
    else:
        pl = np.ascontiguousarray(np.asarray(pair_list, dtype=np.int32).reshape(-1, 2))
        npairs = len(pl)
    if stats is not None:
        if (not stats.is_cuda or stats.dtype != torch.float64 or tuple(stats.shape) != (npairs, 4)
                or not stats.is_contiguous()):
            raise ValueError("stats must be a contiguous (npairs, 4) float64 CUDA tensor")
    if out is None:
        out = torch.empty((npairs, 2), dtype=torch.float64, device=X.device)
    pp = pl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if pl is not None else None
    dev = X.device.index or 0
    rc = load_library().micx_pearson(context(dev), ctypes.c_void_p(X.data_ptr()), dt,
                                     m, n, pp, npairs,
                                     ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check(rc, "micx_pearson")
    _check(status(dev), "micx_pearson")
    return out


def batch(data, off_x, off_y, ns, alphas, cs, mode: int = MODE_FP64, out=None, stream=None,
          wait: bool = True):
    """Independent pairs of uneven n and (alpha, c) from a packed 1-D CUDA
    tensor `data` (float32/float64/int32): pair k is data[off_x[k]:+ns[k]]
    against data[off_y[k]:+ns[k]] with parameters (alphas[k], cs[k]).
    Returns an (npairs, 4) float64 CUDA tensor of (MIC, MAS, MEV, MCN)."""
    import torch
    if not data.is_cuda or data.dim() != 1:
        raise ValueError("data must be a 1-D CUDA tensor")
    data = data.contiguous()
    dt = _DTYPES.get(str(data.dtype))
    if dt is None:
        raise ValueError("data dtype must be float32, float64 or int32")
    off_x, off_y, ns = (np.asarray(a, dtype=np.int64).ravel() for a in (off_x, off_y, ns))
    alphas, cs = (np.asarray(a, dtype=np.float64).ravel() for a in (alphas, cs))
    npairs = len(ns)
    if not (len(off_x) == len(off_y) == len(alphas) == len(cs) == npairs) or npairs < 1:
        raise ValueError("descriptor arrays must be non-empty and of one length")
    if ((off_x + ns) > data.numel()).any() or ((off_y + ns) > data.numel()).any():
        raise ValueError("a pair reaches past the end of data")
    descs = (_PairDesc * npairs)()
    for k in range(npairs):
        descs[k] = _PairDesc(int(off_x[k]), int(off_y[k]), int(ns[k]), 0, float(alphas[k]), float(cs[k]))
    if out is None:
        out = torch.empty((npairs, 4), dtype=torch.float64, device=data.device)
    dev = data.device.index or 0
    rc = load_library().micx_batch(context(dev), ctypes.c_void_p(data.data_ptr()),
                                   dt, descs, npairs, int(mode), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream))
    _check(rc, "micx_batch")
    if wait:
        _check(status(dev), "micx_batch")
    return out


def master(X, i: int, alpha: float = 0.6, c: float = 15.0, mode: int = MODE_FP64, out=None,
           stream=None):
    """One variable against all others (the paper's master-variable mode):
    rows (i, j) of X for every j != i, in increasing j, through micx_pairs.
    Returns an (m-1, 4) float64 CUDA tensor of (MIC, MAS, MEV, MCN)."""
    m = X.shape[0]
    if not 0 <= i < m:
        raise ValueError("master variable out of range")
    return pairs(X, [(i, j) for j in range(m) if j != i], alpha, c, mode, out, stream)


def score_noalloc(x, y, alpha: float, c: float, mode: int, stats, mats=None, status=None,
                  stream=None):
    """micx_score_noalloc: the score of one pair of 1-D CUDA tensors x, y
    (float32/float64/int32, same length) into caller-owned CUDA tensors:
    stats (4 float64), mats (3*W*W float64: M, Axy, Ayx) or None, status
    (1 int32: the device-side result) or None.  Queued on the stream; no
    allocation.  Returns the host-side return code (raises on error)."""
    if x.dtype != y.dtype or x.numel() != y.numel() or not (x.is_cuda and y.is_cuda):
        raise ValueError("x and y must be CUDA tensors of one dtype and length")
    dt = _DTYPES.get(str(x.dtype))
    if dt is None:
        raise ValueError("dtype must be float32, float64 or int32")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    par = _param(alpha, c)
    rc = load_library().micx_score_noalloc(context(x.device.index or 0), ptr(x), ptr(y), dt, x.numel(),
                                           ctypes.byref(par), int(mode), ptr(stats), ptr(mats),
                                           ptr(status), _stream_ptr(stream))
    _check(rc, "micx_score_noalloc")
    return rc


def debug_item(x, y, alpha: float, c: float, orient: int, ry: int, device: int = 0):
    """Integer stages of one item (see micx_debug_item)."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    yhat, k, K = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rs = np.zeros(ry + 1, dtype=np.int32)
    ends = np.zeros(n, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    prob = _Problem(n, _dptr(x), _dptr(y))
    par = _param(alpha, c)
    _check(load_library().micx_debug_item(context(device), ctypes.byref(prob), ctypes.byref(par),
                                          int(orient), int(ry), ctypes.byref(yhat),
                                          rs.ctypes.data_as(ip), ctypes.byref(k), ctypes.byref(K),
                                          ends.ctypes.data_as(ip)), "micx_debug_item")
    return {"yhat": yhat.value, "row_starts": rs[: yhat.value + 1].copy(), "k": k.value,
            "K": K.value, "ends": ends[: K.value].copy()}


def debug_tables(x, y, alpha: float, c: float, orient: int, ry: int, device: int = 0):
    """Tie-group starts of both variables and the DP's cumulative count table
    of one item (see micx_debug_tables): dict with group_start_x,
    group_start_y (n ints) and counts ((K+1) x yhat)."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    it = debug_item(x, y, alpha, c, orient, ry, device)
    gx = np.zeros(n, dtype=np.int32)
    gy = np.zeros(n, dtype=np.int32)
    N = np.zeros((n + 1) * ry, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    prob = _Problem(n, _dptr(x), _dptr(y))
    par = _param(alpha, c)
    _check(load_library().micx_debug_tables(context(device), ctypes.byref(prob), ctypes.byref(par),
                                            int(orient), int(ry), gx.ctypes.data_as(ip),
                                            gy.ctypes.data_as(ip), N.ctypes.data_as(ip)),
           "micx_debug_tables")
    K, yh = it["K"], it["yhat"]
    return {"group_start_x": gx, "group_start_y": gy, "counts": N[: (K + 1) * yh].reshape(K + 1, yh).copy()}


def set_profiling(enable: bool = True, device: int = 0):
    """Record DP kernel time (HIP events) and algorithmic work in pair calls."""
    _check(load_library().micx_set_profiling(context(device), 1 if enable else 0),
           "micx_set_profiling")


def get_profile(device: int = 0) -> dict:
    """Totals of the last pair call: items, dp_cells, h_evals, h_terms, dp_ms, dp_launches."""
    p = _Profile()
    _check(load_library().micx_get_profile(context(device), ctypes.byref(p)), "micx_get_profile")
    return {k: getattr(p, k) for k, _ in _Profile._fields_}


def dp32_bound(n: int, x: int, y: int) -> float:
    """A-priori |dM| bound of the 32-bit DP form for the entries M[l][y],
    l <= x, at sample count n (host arithmetic; no device needed)."""
    return float(load_library().micx_dp32_bound(int(n), int(x), int(y)))


def set_dp32_tolerance(tol: float, device: int = 0):
    """Largest |dM| allowed for a row count to run the DP in 32-bit fixed point."""
    _check(load_library().micx_set_dp32_tolerance(context(device), float(tol)),
           "micx_set_dp32_tolerance")


def set_compat(flags: int, device: int = 0):
    """Compatibility variants (COMPAT_* OR-ed) for every later call on the device."""
    _check(load_library().micx_set_compat(context(device), int(flags)), "micx_set_compat")
