"""Pins for the oracle's exact sums (Sec. I, eqs. 2d1 and 2d2).

Each check is independent of the summation code: closed forms for one point
and one mode, the uniform-grid case where the sums reduce to a textbook DFT
(numpy.fft), the shift theorem, linearity and the adjoint relation.
"""
import math

import numpy as np
import pytest

from oracle import direct, params

R = np.random.default_rng(123)


def _pts(M, dim):
    return tuple(R.uniform(-math.pi, math.pi, M) for _ in range(dim))


def _cplx(shape):
    return R.standard_normal(shape) + 1j * R.standard_normal(shape)


@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("Ns", [(5, 4), (3, 6, 4)])
def test_single_point_closed_form(iflag, Ns):
    dim = len(Ns)
    pts = _pts(1, dim)
    c = _cplx(1)
    f = direct.type1(pts, c, Ns, iflag=iflag)
    ks = np.meshgrid(*[params.mode_indices(N) for N in Ns[::-1]], indexing="ij")
    phase = sum(k * p[0] for k, p in zip(ks[::-1], pts))
    assert np.allclose(f, c[0] * np.exp(iflag * 1j * phase), rtol=0, atol=1e-13)


@pytest.mark.parametrize("iflag", [-1, 1])
def test_single_mode_closed_form(iflag):
    pts = _pts(50, 2)
    Ns = (6, 5)
    f = np.zeros(Ns[::-1], dtype=complex)
    k1, k2 = 2, -2
    f[k2 + Ns[1] // 2, k1 + Ns[0] // 2] = 1.0
    c = direct.type2(pts, f, iflag=iflag)
    assert np.allclose(c, np.exp(iflag * 1j * (k1 * pts[0] + k2 * pts[1])), atol=1e-13)


def _uniform_grid(Ns):
    axes = [-math.pi + 2 * math.pi * np.arange(N) / N for N in Ns]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")      # (N2, N1) / (N3, N2, N1)
    return tuple(m.ravel() for m in mesh[::-1])


def _dft_signed(a, iflag):
    if iflag < 0:
        return np.fft.fftn(a)
    return np.fft.ifftn(a) * a.size


@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("Ns", [(16, 12), (9, 7), (6, 5, 8)])
def test_type1_uniform_grid_is_dft(iflag, Ns):
    """x_j = -pi + 2 pi j/N on a tensor grid: f_k = (-1)^(sum k) DFT(c)[k mod N]."""
    pts = _uniform_grid(Ns)
    c = _cplx(Ns[::-1])
    f = direct.type1(pts, c.ravel(), Ns, iflag=iflag)
    F = _dft_signed(c, iflag)
    idx = [params.mode_indices(N) % N for N in Ns]
    sign = 1.0
    for ax, N in enumerate(Ns[::-1]):
        k = params.mode_indices(N)
        sh = [1] * len(Ns)
        sh[ax] = N
        sign = sign * np.where(k % 2 == 0, 1.0, -1.0).reshape(sh)
    ref = sign * F[np.ix_(*idx[::-1])]
    assert np.allclose(f, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("Ns", [(16, 12), (7, 9, 6)])
def test_type2_uniform_grid_is_dft(iflag, Ns):
    pts = _uniform_grid(Ns)
    f = _cplx(Ns[::-1])
    c = direct.type2(pts, f, iflag=iflag)
    # place (-1)^k f_k at index k mod N, then a plain DFT of sign iflag
    G = np.zeros(Ns[::-1], dtype=complex)
    idx = [params.mode_indices(N) % N for N in Ns]
    sign = 1.0
    for ax, N in enumerate(Ns[::-1]):
        k = params.mode_indices(N)
        sh = [1] * len(Ns)
        sh[ax] = N
        sign = sign * np.where(k % 2 == 0, 1.0, -1.0).reshape(sh)
    G[np.ix_(*idx[::-1])] = sign * f
    ref = _dft_signed(G, iflag).ravel()
    assert np.allclose(c, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_shift_theorem_and_linearity():
    Ns = (7, 6)
    pts = _pts(40, 2)
    c1, c2 = _cplx(40), _cplx(40)
    d = (0.37, -1.1)
    f = direct.type1(pts, c1, Ns, iflag=-1)
    fs = direct.type1((pts[0] + d[0], pts[1] + d[1]), c1, Ns, iflag=-1)
    k2, k1 = np.meshgrid(params.mode_indices(6), params.mode_indices(7), indexing="ij")
    assert np.allclose(fs, f * np.exp(-1j * (k1 * d[0] + k2 * d[1])), atol=1e-12)
    a = 0.3 - 2.0j
    lin = direct.type1(pts, a * c1 + c2, Ns, iflag=-1)
    assert np.allclose(lin, a * f + direct.type1(pts, c2, Ns, iflag=-1), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_of_exact_sums(dim):
    Ns = (5, 6, 4)[:dim]
    pts = _pts(30, dim)
    c = _cplx(30)
    f = _cplx(Ns[::-1])
    lhs = np.vdot(direct.type1(pts, c, Ns, iflag=-1), f)
    rhs = np.vdot(c, direct.type2(pts, f, iflag=+1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_mode_subset_matches_full():
    Ns = (9, 8, 5)
    pts = _pts(25, 3)
    c = _cplx(25)
    full = direct.type1(pts, c, Ns, iflag=1)
    kk = (np.array([-4, 0, 3]), np.array([-4, 2]), np.array([1]))
    sub = direct.type1(pts, c, Ns, iflag=1, kk=kk)
    ref = full[np.ix_(kk[2] + 2, kk[1] + 4, kk[0] + 4)]
    assert np.allclose(sub, ref, atol=1e-13)
    idx = np.array([3, 0, 24])
    f = _cplx(Ns[::-1])
    assert np.allclose(direct.type2(pts, f, idx=idx), direct.type2(pts, f)[idx], atol=1e-13)
