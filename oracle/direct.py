"""Exact exponential sums and plain spreading/interpolation (C/OpenMP, FP64).

Dimensions 1, 2 and 3 are accepted; coordinates are passed as a tuple of d
arrays.

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).  Thin
ctypes wrappers over ``oracle/csrc/oracle.c``; inputs are widened to float64.
"""
import ctypes

import numpy as np

from . import build as _build

_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        _lib.orc_direct_type1.argtypes = [
            ctypes.c_int, ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int,
            ctypes.c_int64, ip, ctypes.c_int64, ip, ctypes.c_int64, ip, dp]
        _lib.orc_direct_type2.argtypes = [
            ctypes.c_int, ip, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int64, ip, dp]
        _lib.orc_spread.argtypes = [
            ctypes.c_int, ip, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
            dp, dp, dp, dp, dp]
        _lib.orc_interp.argtypes = _lib.orc_spread.argtypes
        _lib.orc_direct_type3.argtypes = [
            ctypes.c_int, ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int, dp, dp, dp,
            ctypes.c_int64, ip, dp]
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads():
    return int(_L().orc_num_threads())


def set_threads(n):
    """Threads of the C loops (a timing control; results are unchanged)."""
    _L().orc_set_threads(int(n))


def _xyz(pts):
    """The d coordinate arrays as float64, padded with None up to three."""
    dim = len(pts)
    if dim not in (1, 2, 3):
        raise ValueError("1, 2 or 3 coordinate arrays expected")
    a = [_f64(p) for p in pts] + [None] * (3 - dim)
    return dim, a[0], a[1], a[2]


def _mode_list(N):
    return np.arange(-(N // 2), N - N // 2, dtype=np.int64)


def type1(pts, c, Ns, iflag=-1, kk=None):
    """Exact type 1 sum f_k = sum_j c_j exp(iflag i k.x_j) (Sec. I, eq. 2d1; 3D
    analogue).

    pts: tuple of d coordinate arrays of length M.  c: complex (M,).
    Ns: mode counts (N1, N2[, N3]).  kk: optional tuple of per-dimension integer
    mode lists (a tensor-product subset); default all of I_N1 x I_N2 (x I_N3).
    Returns a complex array of shape (K3, K2, K1) (2D: (K2, K1); 1D: (K1,)),
    k1 fastest.
    """
    dim, x, y, z = _xyz(pts)
    M = x.shape[0]
    if kk is None:
        kk = tuple(_mode_list(N) for N in Ns)
    k1 = np.ascontiguousarray(kk[0], dtype=np.int64)
    k2 = np.ascontiguousarray(kk[1], dtype=np.int64) if dim >= 2 else np.zeros(1, np.int64)
    k3 = np.ascontiguousarray(kk[2], dtype=np.int64) if dim == 3 else np.zeros(1, np.int64)
    c = _c128(c)
    out = np.zeros(len(k1) * len(k2) * len(k3), dtype=np.complex128)
    _L().orc_direct_type1(dim, M, _dp(x), _dp(y), _dp(z), _dp(c.view(np.float64)),
                          int(iflag), len(k1), _ip(k1), len(k2), _ip(k2),
                          len(k3), _ip(k3), _dp(out.view(np.float64)))
    shape = ((len(k1),), (len(k2), len(k1)), (len(k3), len(k2), len(k1)))[dim - 1]
    return out.reshape(shape)


def type2(pts, f, iflag=+1, idx=None):
    """Exact type 2 sum c_j = sum_k f_k exp(iflag i k.x_j) (Sec. I, eq. 2d2).

    f: complex array of shape (N1,), (N2, N1) or (N3, N2, N1), k1 fastest, modes in
    ascending order from -floor(N/2).  idx: optional indices of the targets
    to evaluate (default all).  Returns complex (len(idx),).
    """
    dim, x, y, z = _xyz(pts)
    f = _c128(f)
    Ns = np.array(list(f.shape[::-1]) + [1] * (3 - f.ndim), dtype=np.int64)
    if idx is None:
        idx = np.arange(x.shape[0], dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(len(idx), dtype=np.complex128)
    _L().orc_direct_type2(dim, _ip(Ns), _dp(x), _dp(y), _dp(z), _dp(f.view(np.float64)),
                          int(iflag), len(idx), _ip(idx), _dp(out.view(np.float64)))
    return out


def spread(pts, c, ns, w, beta):
    """Fine grid b_l = sum_j c_j psi_per(l h - pi - x_j) (Sec. II-A step 1).

    Returns complex (n1,), (n2, n1) or (n3, n2, n1), first coordinate fastest."""
    dim, x, y, z = _xyz(pts)
    c = _c128(c)
    nn = np.array(list(ns) + [1] * (3 - dim), dtype=np.int64)
    grid = np.zeros(int(np.prod(ns)), dtype=np.complex128)
    _L().orc_spread(dim, _ip(nn), int(w), float(beta), x.shape[0], _dp(x), _dp(y), _dp(z),
                    _dp(c.view(np.float64)), _dp(grid.view(np.float64)))
    return grid.reshape(tuple(ns[::-1]))


def interp(pts, grid, w, beta):
    """c_j = sum_l b_l psi_per(l h - pi - x_j) (Sec. II-B step 3)."""
    dim, x, y, z = _xyz(pts)
    grid = _c128(grid)
    ns = grid.shape[::-1]
    nn = np.array(list(ns) + [1] * (3 - dim), dtype=np.int64)
    c = np.zeros(x.shape[0], dtype=np.complex128)
    _L().orc_interp(dim, _ip(nn), int(w), float(beta), x.shape[0], _dp(x), _dp(y), _dp(z),
                    _dp(grid.view(np.float64)), _dp(c.view(np.float64)))
    return c


def type3(pts, c, freqs, iflag=-1, idx=None):
    """Exact type 3 sum f_k = sum_j c_j exp(iflag i s_k.x_j) at real
    frequencies s_k (the transform named in Sec. I-B and Sec. VI as outside
    the paper's scope).

    pts: d coordinate arrays of length M (any real values).  freqs: d arrays
    of length K.  idx: optional indices of the frequencies to evaluate
    (default all).  Returns complex (len(idx),)."""
    dim, x, y, z = _xyz(pts)
    dk, s, t, u = _xyz(freqs)
    if dk != dim:
        raise ValueError("points and frequencies differ in dimension")
    c = _c128(c)
    if idx is None:
        idx = np.arange(s.shape[0], dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(len(idx), dtype=np.complex128)
    _L().orc_direct_type3(dim, x.shape[0], _dp(x), _dp(y), _dp(z), _dp(c.view(np.float64)),
                          int(iflag), _dp(s), _dp(t), _dp(u), len(idx), _ip(idx),
                          _dp(out.view(np.float64)))
    return out
