"""FP64 CPU oracle for the MINE characteristic matrix and statistics.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library (``paper_1208_4271_amd``) never imports, links or calls it, and the two
share no code: the only module both sides use is ``workloads`` (seeded input
generators, no arithmetic of the method).

The computation lives in ``mine_oracle.c`` (plain C, FP64, libm ``log``); this
module compiles it with gcc and exposes it through ctypes with numpy arrays.
The paper passages each step follows are cited in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mine_oracle.c")
_LIB = os.path.join(_HERE, "libmine_oracle.so")

# Reading flags (same bit values as in mine_oracle.c).
TIE_STRICT = 1
DESIRED_INT = 2
COMBINE_INDEX = 4
NORM_BY_Y = 8
BOUND_STRICT = 16
KHAT_PLUS1 = 32

from .pearson import nonlinearity, pearson  # noqa: E402,F401  (Pearson's rho, MIC - rho^2)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libmine_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _use_library:
    """Context manager: temporarily route every call to another build of the
    oracle (used by the mutation tests, which compile deliberately broken
    copies of mine_oracle.c to show that the pins catch them)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = None
        lib = ctypes.CDLL(self.path)
        _lib = _configure(lib)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(lib):
    P = ctypes.POINTER
    dp, ip = P(ctypes.c_double), P(ctypes.c_int)
    lib.oracle_grid_bound.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.oracle_grid_bound.restype = ctypes.c_int
    lib.oracle_grid_width.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_grid_width.restype = ctypes.c_int
    lib.oracle_equipartition.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_equipartition.restype = ctypes.c_int
    lib.oracle_clumps.argtypes = [dp, ip, ctypes.c_int, ip]
    lib.oracle_clumps.restype = ctypes.c_int
    lib.oracle_superclumps.argtypes = [dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip]
    lib.oracle_superclumps.restype = ctypes.c_int
    lib.oracle_optimize_x_axis.argtypes = [ip, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, dp, ip]
    lib.oracle_optimize_x_axis.restype = ctypes.c_int
    lib.oracle_score.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_score.restype = ctypes.c_int
    lib.oracle_item.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip]
    lib.oracle_item.restype = ctypes.c_int
    lib.oracle_counts.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_counts.restype = ctypes.c_int
    lib.oracle_group_starts.argtypes = [dp, ctypes.c_int, ip]
    lib.oracle_group_starts.restype = None
    lib.oracle_allpairs.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, P(ctypes.c_longlong),
                                    ctypes.c_longlong, ctypes.c_int, dp]
    lib.oracle_allpairs.restype = ctypes.c_int
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid_bound(n: int, alpha: float) -> int:
    """floor(n ** alpha) in FP64 (Sec. 2C; Appendix A item 1)."""
    return _load().oracle_grid_bound(int(n), float(alpha))


def grid_width(n: int, alpha: float, flags: int = 0) -> int:
    """Side W of the dense matrices returned by :func:`score`."""
    return _load().oracle_grid_width(int(n), float(alpha), int(flags))


def equipartition(v_sorted, y: int, flags: int = 0):
    """EquipartitionYAxis on ascending values: (rows per point, yhat)."""
    v = _f64(v_sorted)
    q = np.zeros(len(v), dtype=np.int32)
    yhat = _load().oracle_equipartition(_dptr(v), len(v), int(y), int(flags), _iptr(q))
    return q, yhat


def clumps(a_sorted, q):
    """GetClumpsPartition: (clump per point, k)."""
    a = _f64(a_sorted)
    q = np.ascontiguousarray(q, dtype=np.int32)
    p = np.zeros(len(a), dtype=np.int32)
    k = _load().oracle_clumps(_dptr(a), _iptr(q), len(a), _iptr(p))
    return p, k


def superclumps(a_sorted, q, khat: int, flags: int = 0):
    """GetSuperclumpsPartition: (superclump per point, K, k)."""
    a = _f64(a_sorted)
    q = np.ascontiguousarray(q, dtype=np.int32)
    p = np.zeros(len(a), dtype=np.int32)
    k = ctypes.c_int(0)
    K = _load().oracle_superclumps(_dptr(a), _iptr(q), len(a), int(khat), int(flags),
                                   _iptr(p), ctypes.byref(k))
    return p, K, k.value


def optimize_x_axis(col, row, K: int, yhat: int, x: int):
    """OptimizeXAxis: (I_l for l = 2..x in nats, column ends of each optimum)."""
    col = np.ascontiguousarray(col, dtype=np.int32)
    row = np.ascontiguousarray(row, dtype=np.int32)
    I = np.zeros(x - 1, dtype=np.float64)
    cuts = np.zeros((x - 1) * x, dtype=np.int32)
    rc = _load().oracle_optimize_x_axis(_iptr(col), _iptr(row), len(col), int(K), int(yhat),
                                        int(x), _dptr(I), _iptr(cuts))
    if rc != 0:
        raise ValueError("oracle_optimize_x_axis: bad arguments")
    return I, cuts.reshape(x - 1, x)


def score(x, y, alpha: float = 0.6, c: float = 15.0, flags: int = 0):
    """Whole score of one pair.

    Returns a dict with ``stats`` = (MIC, MAS, MEV, MCN), ``M`` (W x W,
    ``M[yy-2, xx-2]`` = M_{xx,yy}, NaN outside xx*yy <= B), ``Axy`` and ``Ayx``
    (per-orientation normalised scores, same layout: [rows-2, cols-2]).
    """
    x, y = _f64(x), _f64(y)
    n = len(x)
    if len(y) != n:
        raise ValueError("x and y differ in length")
    W = grid_width(n, alpha, flags)
    if W < 1:
        raise ValueError("grid bound below 4: no cell")
    M = np.zeros(W * W)
    Axy = np.zeros(W * W)
    Ayx = np.zeros(W * W)
    st = np.zeros(4)
    rc = _load().oracle_score(_dptr(x), _dptr(y), n, float(alpha), float(c), int(flags),
                              _dptr(M), _dptr(Axy), _dptr(Ayx), _dptr(st))
    if rc != 0:
        raise ValueError("oracle_score: bad arguments")
    lim = grid_bound(n, alpha) - (1 if flags & BOUND_STRICT else 0)
    mask = np.zeros((W, W), dtype=bool)
    for r in range(2, W + 2):
        for cc in range(2, W + 2):
            mask[r - 2, cc - 2] = r * cc <= lim
    M = M.reshape(W, W)
    Axy = Axy.reshape(W, W)
    Ayx = Ayx.reshape(W, W)
    M[~mask] = np.nan
    Axy[~mask] = np.nan
    Ayx[~mask] = np.nan
    return {"stats": st, "M": M, "Axy": Axy, "Ayx": Ayx, "B": lim, "W": W}


def item(x, y, alpha: float, c: float, orient: int, ry: int, flags: int = 0):
    """Integer stages of one (orientation, row count) item."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    yhat, k, K = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    rs = np.zeros(ry + 1, dtype=np.int32)
    ends = np.zeros(n, dtype=np.int32)
    rc = _load().oracle_item(_dptr(x), _dptr(y), n, float(alpha), float(c), int(flags),
                             int(orient), int(ry), ctypes.byref(yhat), _iptr(rs),
                             ctypes.byref(k), ctypes.byref(K), _iptr(ends))
    if rc != 0:
        raise ValueError("oracle_item: bad arguments")
    return {"yhat": yhat.value, "row_starts": rs[: yhat.value + 1].copy(), "k": k.value,
            "K": K.value, "ends": ends[: K.value].copy()}


def counts(x, y, alpha: float, c: float, orient: int, ry: int, flags: int = 0):
    """Cumulative count table of one item (App. A item 10a): int array
    (K+1, yhat), row t = points of the first t superclumps per row."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    N = np.zeros((n + 1) * ry, dtype=np.int32)
    K = _load().oracle_counts(_dptr(x), _dptr(y), n, float(alpha), float(c), int(flags), int(orient),
                              int(ry), _iptr(N))
    if K < 0:
        raise ValueError("oracle_counts: bad arguments")
    yh = item(x, y, alpha, c, orient, ry, flags)["yhat"]
    return N[: (K + 1) * yh].reshape(K + 1, yh).copy()


def group_starts(v):
    """Sorted position where each sample's tie group starts (count of
    smaller values)."""
    v = _f64(v)
    out = np.zeros(len(v), dtype=np.int32)
    _load().oracle_group_starts(_dptr(v), len(v), _iptr(out))
    return out


def allpairs(X, alpha: float = 0.6, c: float = 15.0, pairs=None, nthreads: int | None = None,
             flags: int = 0):
    """Statistics of many pairs of rows of X (m x n): array (npairs, 4)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    if pairs is None:
        npairs = m * (m - 1) // 2
        pp = None
    else:
        pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
        npairs = len(pairs)
        pp = pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))
    out = np.zeros((npairs, 4))
    rc = _load().oracle_allpairs(_dptr(X), m, n, float(alpha), float(c), int(flags), pp,
                                 npairs, int(nthreads), _dptr(out))
    if rc != 0:
        raise ValueError("oracle_allpairs: bad arguments")
    return out
