"""Reference gradients of the exact type 1 and type 2 sums (FP64).

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).

Complex gradients follow the convention g = dL/dRe(z) + i dL/dIm(z) for a real
loss L, so that dL = Re(conj(g) dz).

Type 2, c = A f with A_jk = exp(s i k.x_j) (Sec. I, eq. 2d2):
  grad_f = A^H g_c                         (the type 1 sum with sign -s)
  grad_x_{j,i} = Re(conj(g_j) sum_k f_k (s i k_i) exp(s i k.x_j))
Type 1, f = A c with A_kj = exp(s i k.x_j) (Sec. I, eq. 2d1):
  grad_c = A^H g_f                         (the type 2 sum with sign -s)
  grad_x_{j,i} = Re(conj(c_j) sum_k g_k (-s i k_i) exp(-s i k.x_j))
Each derivative sum is an exact type 2 sum with coefficients multiplied by
(+-s i k_i), evaluated by ``direct.type2``.
"""
import numpy as np

from . import direct, params


def _ki_weight(shape, axis_from_fastest):
    """k_i for every mode of an array shaped (..., N2, N1)."""
    N = shape[-1 - axis_from_fastest]
    k = params.mode_indices(N).astype(np.float64)
    sh = [1] * len(shape)
    sh[-1 - axis_from_fastest] = N
    return k.reshape(sh)


def type2_grad_f(pts, f_shape, g, iflag=+1):
    """grad_f = A^H g for c = type2(f): the exact type 1 sum with sign -iflag."""
    return direct.type1(pts, g, tuple(f_shape)[::-1], iflag=-iflag)


def type2_grad_x(pts, f, g, iflag=+1, idx=None):
    """grad_x for c = type2(f) with upstream g, at the indices idx (default all):
    Re(conj(g_j) sum_k f_k (s i k_i) exp(s i k.x_j)) per dimension i."""
    dim = len(pts)
    f = np.asarray(f, dtype=np.complex128)
    if idx is None:
        idx = np.arange(len(pts[0]))
    gx = []
    for i in range(dim):
        fi = f * (iflag * 1j) * _ki_weight(f.shape, i)
        dc = direct.type2(pts, fi, iflag=iflag, idx=idx)
        gx.append(np.real(np.conj(np.asarray(g)[idx]) * dc))
    return gx


def type2_grads(pts, f, g, iflag=+1, idx=None):
    """(grad_f, grad_x list) for c = type2(f) with upstream g (length M).
    grad_x is evaluated at the indices idx (default all points)."""
    f = np.asarray(f, dtype=np.complex128)
    return type2_grad_f(pts, f.shape, g, iflag), type2_grad_x(pts, f, g, iflag, idx)


def type1_grads(pts, c, Ns, gf, iflag=-1, idx=None):
    """(grad_c, grad_x list) for f = type1(c) with upstream gf shaped like f."""
    dim = len(pts)
    gf = np.asarray(gf, dtype=np.complex128)
    if idx is None:
        idx = np.arange(len(pts[0]))
    grad_c = direct.type2(pts, gf, iflag=-iflag, idx=idx)
    gx = []
    for i in range(dim):
        gi = gf * (-iflag * 1j) * _ki_weight(gf.shape, i)
        d = direct.type2(pts, gi, iflag=-iflag, idx=idx)
        gx.append(np.real(np.conj(np.asarray(c)[idx]) * d))
    return grad_c, gx
