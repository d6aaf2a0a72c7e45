"""Oracle for distance reporting along a space-filling curve.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product library never does.  It
shares no code with the HIP path.

The arithmetic lives in ``sfc_oracle.cpp`` (plain C++, built with g++ and
``-ffp-contract=off``); this module is a ctypes wrapper around it plus the
learned-index reference in :mod:`oracle.learned`.  Every function cites the
passage of the paper it follows in the C++ source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfc_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

MORTON = 0
HILBERT = 1
L2 = 0       # closed Euclidean ball of radius delta
LINF = 1     # closed axis-parallel square window of half side delta


def compile_lib() -> str:
    """Compile the oracle with g++ (host only, no fused multiply-add)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-pthread", _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            compile_lib()
        L = ctypes.CDLL(_LIB)
        u64, u32, i32, i64, dbl, vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_double, ctypes.c_void_p)
        L.oracle_morton.argtypes = [u32, u32]
        L.oracle_morton.restype = u64
        L.oracle_hilbert.argtypes = [u32, u32]
        L.oracle_hilbert.restype = u64
        L.oracle_quantize.argtypes = [vp, u64, vp, vp]
        L.oracle_quantize.restype = i32
        L.oracle_keys.argtypes = [vp, u64, i32, vp]
        L.oracle_keys.restype = i32
        L.oracle_build.argtypes = [vp, u64, i32, vp, vp, vp]
        L.oracle_build.restype = i32
        L.oracle_box.argtypes = [dbl, dbl, dbl, vp]
        L.oracle_box.restype = i32
        L.oracle_ranges.argtypes = [dbl, dbl, dbl, i32, vp, vp]
        L.oracle_ranges.restype = i32
        L.oracle_box_ranges.argtypes = [i64, i64, i64, i64, i32, vp, vp]
        L.oracle_box_ranges.restype = i32
        L.oracle_index_ranges.argtypes = [vp, u64, dbl, dbl, dbl, i32, vp]
        L.oracle_index_ranges.restype = i32
        L.oracle_query.argtypes = [vp, vp, vp, u64, vp, vp, u64, i32, vp, vp, u64, i32, i32]
        L.oracle_query.restype = i64
        L.oracle_brute.argtypes = [vp, u64, vp, vp, u64, vp, vp, u64, i32]
        L.oracle_brute.restype = i64
        L.oracle_morton3.argtypes = [u32, u32, u32]
        L.oracle_morton3.restype = u64
        L.oracle_keys3.argtypes = [vp, u64, vp]
        L.oracle_keys3.restype = i32
        L.oracle_build3.argtypes = [vp, u64, vp, vp, vp]
        L.oracle_build3.restype = i32
        L.oracle_box3.argtypes = [vp, dbl, vp]
        L.oracle_box3.restype = i32
        L.oracle_ranges3.argtypes = [vp, dbl, vp, vp]
        L.oracle_ranges3.restype = i32
        L.oracle_box_ranges3.argtypes = [vp, vp, vp]
        L.oracle_box_ranges3.restype = i32
        L.oracle_query3.argtypes = [vp, vp, vp, u64, vp, vp, u64, vp, vp, u64, i32, i32]
        L.oracle_query3.restype = i64
        L.oracle_brute3.argtypes = [vp, u64, vp, vp, u64, vp, vp, u64, i32]
        L.oracle_brute3.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _xy(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 2:
        raise ValueError("expected an (n, 2) array of float64")
    return a


class DomainError(ValueError):
    pass


class InvalidQuery(ValueError):
    pass


def morton(x: int, y: int) -> int:
    return int(lib().oracle_morton(x, y))


def hilbert(x: int, y: int) -> int:
    return int(lib().oracle_hilbert(x, y))


def key(curve: int, x: int, y: int) -> int:
    return morton(x, y) if curve == MORTON else hilbert(x, y)


def quantize(xy):
    xy = _xy(xy)
    n = xy.shape[0]
    ux = np.empty(n, np.uint32)
    uy = np.empty(n, np.uint32)
    if lib().oracle_quantize(_p(xy), n, _p(ux), _p(uy)) != 0:
        raise DomainError("coordinate outside [0,1)")
    return ux, uy


def keys(xy, curve: int) -> np.ndarray:
    xy = _xy(xy)
    out = np.empty(xy.shape[0], np.uint64)
    if lib().oracle_keys(_p(xy), xy.shape[0], curve, _p(out)) != 0:
        raise DomainError("coordinate outside [0,1)")
    return out


def build(xy, curve: int):
    """Sorted (keys u64, ids u32, xy f64[n,2]) of the construction."""
    xy = _xy(xy)
    n = xy.shape[0]
    k = np.empty(n, np.uint64)
    i = np.empty(n, np.uint32)
    s = np.empty((n, 2), np.float64)
    if lib().oracle_build(_p(xy), n, curve, _p(k), _p(i), _p(s)) != 0:
        raise DomainError("coordinate outside [0,1)")
    return k, i, s


def box(qx: float, qy: float, delta: float):
    """Widened integer box (lo_x, hi_x, lo_y, hi_y), or None when empty."""
    b = np.zeros(4, np.int64)
    r = lib().oracle_box(qx, qy, delta, _p(b))
    if r < 0:
        raise InvalidQuery("invalid query")
    return tuple(int(v) for v in b) if r == 1 else None


def ranges(qx: float, qy: float, delta: float, curve: int):
    """Merged key ranges [(lo, hi), ...] (inclusive), at most four."""
    lo = np.zeros(4, np.uint64)
    hi = np.zeros(4, np.uint64)
    k = lib().oracle_ranges(qx, qy, delta, curve, _p(lo), _p(hi))
    if k < 0:
        raise InvalidQuery("invalid query")
    return [(int(lo[i]), int(hi[i])) for i in range(k)]


def box_ranges(lx: int, hx: int, ly: int, hy: int, curve: int):
    """Merged key ranges of cells(Q) for an integer box (inclusive bounds)."""
    lo = np.zeros(4, np.uint64)
    hi = np.zeros(4, np.uint64)
    k = lib().oracle_box_ranges(lx, hx, ly, hy, curve, _p(lo), _p(hi))
    if k < 0:
        raise ValueError("box outside the domain")
    return [(int(lo[i]), int(hi[i])) for i in range(k)]


def index_ranges(sorted_keys, qx: float, qy: float, delta: float, curve: int):
    sk = np.ascontiguousarray(sorted_keys, np.uint64)
    be = np.zeros(8, np.uint64)
    k = lib().oracle_index_ranges(_p(sk), sk.shape[0], qx, qy, delta, curve, _p(be))
    if k < 0:
        raise InvalidQuery("invalid query")
    return [(int(be[2 * i]), int(be[2 * i + 1])) for i in range(k)]


def query(index, q, delta, curve: int, nthreads: int = 1, metric: int = L2):
    """CSR (offsets u64[m+1], ids u32[total]) of a query batch over a built
    index (the tuple returned by :func:`build`).  metric L2: the ball of
    radius delta; LINF: the square window of half side delta."""
    sk, si, sxy = index
    sk = np.ascontiguousarray(sk, np.uint64)
    si = np.ascontiguousarray(si, np.uint32)
    sxy = _xy(sxy)
    q = _xy(q)
    d = np.ascontiguousarray(delta, np.float64)
    m = q.shape[0]
    if d.shape != (m,):
        raise ValueError("delta must have one entry per query")
    off = np.zeros(m + 1, np.uint64)
    L = lib()
    tot = L.oracle_query(_p(sk), _p(si), _p(sxy), sk.shape[0], _p(q), _p(d), m, curve,
                         _p(off), None, 0, nthreads, metric)
    if tot < 0:
        raise InvalidQuery("invalid query")
    ids = np.zeros(max(int(tot), 1), np.uint32)
    L.oracle_query(_p(sk), _p(si), _p(sxy), sk.shape[0], _p(q), _p(d), m, curve,
                   _p(off), _p(ids), int(tot), nthreads, metric)
    return off, ids[: int(tot)]


def brute(xy, q, delta, metric: int = L2):
    """Brute-force CSR (ids ascending per query), same test as :func:`query`."""
    xy = _xy(xy)
    q = _xy(q)
    d = np.ascontiguousarray(delta, np.float64)
    m = q.shape[0]
    off = np.zeros(m + 1, np.uint64)
    L = lib()
    tot = L.oracle_brute(_p(xy), xy.shape[0], _p(q), _p(d), m, _p(off), None, 0, metric)
    if tot < 0:
        raise InvalidQuery("invalid query")
    ids = np.zeros(max(int(tot), 1), np.uint32)
    L.oracle_brute(_p(xy), xy.shape[0], _p(q), _p(d), m, _p(off), _p(ids), int(tot), metric)
    return off, ids[: int(tot)]


def canonical(offsets, ids):
    """Sorted (query, id) pairs of a CSR result, as one int64 array of
    query * 2^32 + id (the canonical comparison form)."""
    offsets = np.asarray(offsets, np.int64)
    ids = np.asarray(ids, np.int64)
    m = offsets.shape[0] - 1
    qidx = np.repeat(np.arange(m, dtype=np.int64), np.diff(offsets))
    return np.sort(qidx * (1 << 32) + ids[: offsets[-1]])


# ---- three dimensions (d = 3 Morton codes) ------------------------------------


def _xyz(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("expected an (n, 3) array of float64")
    return a


def morton3(x: int, y: int, z: int) -> int:
    return int(lib().oracle_morton3(x, y, z))


def keys3(xyz) -> np.ndarray:
    xyz = _xyz(xyz)
    k = np.zeros(xyz.shape[0], np.uint64)
    if lib().oracle_keys3(_p(xyz), xyz.shape[0], _p(k)) != 0:
        raise DomainError("coordinate outside [0,1)")
    return k


def build3(xyz):
    """(sorted keys u64, ids u32, points f64 (n, 3)) of a 3-D point set."""
    xyz = _xyz(xyz)
    n = xyz.shape[0]
    k = np.zeros(n, np.uint64)
    i = np.zeros(n, np.uint32)
    s = np.zeros((n, 3), np.float64)
    if lib().oracle_build3(_p(xyz), n, _p(k), _p(i), _p(s)) != 0:
        raise DomainError("coordinate outside [0,1)")
    return k, i, s


def box3(q, delta: float):
    """Widened integer box (lx, hx, ly, hy, lz, hz), or None when empty."""
    qq = np.ascontiguousarray(q, np.float64)
    b = np.zeros(6, np.int64)
    r = lib().oracle_box3(_p(qq), delta, _p(b))
    if r < 0:
        raise InvalidQuery("invalid query")
    return tuple(int(v) for v in b) if r == 1 else None


def ranges3(q, delta: float):
    """Merged key ranges [(lo, hi), ...] (inclusive) of a 3-D query, at most 8."""
    qq = np.ascontiguousarray(q, np.float64)
    lo = np.zeros(8, np.uint64)
    hi = np.zeros(8, np.uint64)
    k = lib().oracle_ranges3(_p(qq), delta, _p(lo), _p(hi))
    if k < 0:
        raise InvalidQuery("invalid query")
    return [(int(lo[i]), int(hi[i])) for i in range(k)]


def box_ranges3(box):
    b = np.ascontiguousarray(box, np.int64)
    lo = np.zeros(8, np.uint64)
    hi = np.zeros(8, np.uint64)
    k = lib().oracle_box_ranges3(_p(b), _p(lo), _p(hi))
    if k < 0:
        raise ValueError("box outside the domain")
    return [(int(lo[i]), int(hi[i])) for i in range(k)]


def query3(index, q, delta, nthreads: int = 1, metric: int = L2):
    """CSR (offsets u64[m+1], ids u32[total]) of 3-D queries over build3's
    output: ball of radius delta (L2) or cube of half side delta (LINF)."""
    sk, si, sxyz = index
    sk = np.ascontiguousarray(sk, np.uint64)
    si = np.ascontiguousarray(si, np.uint32)
    sxyz = _xyz(sxyz)
    q = _xyz(q)
    d = np.ascontiguousarray(delta, np.float64)
    m = q.shape[0]
    if d.shape != (m,):
        raise ValueError("delta must have one entry per query")
    off = np.zeros(m + 1, np.uint64)
    L = lib()
    tot = L.oracle_query3(_p(sk), _p(si), _p(sxyz), sk.shape[0], _p(q), _p(d), m, _p(off), None,
                          0, nthreads, metric)
    if tot < 0:
        raise InvalidQuery("invalid query")
    ids = np.zeros(max(int(tot), 1), np.uint32)
    L.oracle_query3(_p(sk), _p(si), _p(sxyz), sk.shape[0], _p(q), _p(d), m, _p(off), _p(ids),
                    int(tot), nthreads, metric)
    return off, ids[: int(tot)]


def brute3(xyz, q, delta, metric: int = L2):
    xyz = _xyz(xyz)
    q = _xyz(q)
    d = np.ascontiguousarray(delta, np.float64)
    m = q.shape[0]
    off = np.zeros(m + 1, np.uint64)
    L = lib()
    tot = L.oracle_brute3(_p(xyz), xyz.shape[0], _p(q), _p(d), m, _p(off), None, 0, metric)
    if tot < 0:
        raise InvalidQuery("invalid query")
    ids = np.zeros(max(int(tot), 1), np.uint32)
    L.oracle_brute3(_p(xyz), xyz.shape[0], _p(q), _p(d), m, _p(off), _p(ids), int(tot), metric)
    return off, ids[: int(tot)]
