"""Pins for the oracle's three-step algorithm (Sec. II) against the exact sums
and against properties that hold exactly (transposition, kernel footprint)."""
import math

import numpy as np
import pytest

from oracle import direct, nufft, params

R = np.random.default_rng(7)


def _pts(M, dim):
    return tuple(R.uniform(-math.pi, math.pi, M) for _ in range(dim))


def _cplx(shape):
    return R.standard_normal(shape) + 1j * R.standard_normal(shape)


CASES = [
    ((16, 12), 1e-2), ((16, 12), 1e-5), ((17, 10), 1e-9), ((12, 13), 1e-12),
    ((8, 10, 6), 1e-5), ((7, 8, 9), 1e-9),
]


@pytest.mark.parametrize("Ns,eps", CASES)
@pytest.mark.parametrize("iflag", [-1, 1])
def test_type1_matches_direct_sum(Ns, eps, iflag):
    pts = _pts(300, len(Ns))
    c = _cplx(300)
    got = nufft.type1(pts, c, Ns, eps, iflag=iflag)
    ref = direct.type1(pts, c, Ns, iflag=iflag)
    assert nufft.rel_l2(got, ref) <= 10 * eps


@pytest.mark.parametrize("Ns,eps", CASES)
@pytest.mark.parametrize("iflag", [-1, 1])
def test_type2_matches_direct_sum(Ns, eps, iflag):
    pts = _pts(300, len(Ns))
    f = _cplx(Ns[::-1])
    got = nufft.type2(pts, f, eps, iflag=iflag)
    ref = direct.type2(pts, f, iflag=iflag)
    assert nufft.rel_l2(got, ref) <= 10 * eps


def test_type1_points_outside_period():
    """Points in [-3pi, 3pi) are folded; the sums are 2pi-periodic in x."""
    Ns = (10, 8)
    pts = _pts(200, 2)
    shifted = (pts[0] + 2 * math.pi * R.integers(-1, 2, 200), pts[1] - 2 * math.pi)
    c = _cplx(200)
    ref = direct.type1(pts, c, Ns)
    assert nufft.rel_l2(nufft.type1(shifted, c, Ns, 1e-6), ref) <= 1e-5


@pytest.mark.parametrize("dim,eps", [(2, 1e-5), (3, 1e-3), (2, 1e-12)])
@pytest.mark.parametrize("iflag", [-1, 1])
def test_adjoint_identity_to_rounding(dim, eps, iflag):
    """<T1 c, f> = <c, T2 f> for the approximate operators too: the steps of
    type 2 (sign -s) are the exact transposes of those of type 1 (sign s)."""
    Ns = (12, 10, 6)[:dim]
    pts = _pts(250, dim)
    c = _cplx(250)
    f = _cplx(Ns[::-1])
    lhs = np.vdot(nufft.type1(pts, c, Ns, eps, iflag=iflag), f)
    rhs = np.vdot(c, nufft.type2(pts, f, eps, iflag=-iflag))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(c) * np.linalg.norm(f) * 10


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_is_transpose_of_interp(dim):
    P = nufft.Params((8, 6, 5)[:dim], 1e-4)
    pts = _pts(100, dim)
    c = _cplx(100)
    b = _cplx(P.ns[::-1])
    lhs = np.vdot(direct.spread(pts, c, P.ns, P.w, P.beta), b)
    rhs = np.vdot(c, direct.interp(pts, b, P.w, P.beta))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) * 10


@pytest.mark.parametrize("w", [2, 5, 6])
def test_spread_single_point_footprint(w):
    """Brute force over every cell: a point puts phi(2 d / w) on the cells at
    signed periodic distance d in [-w/2, w/2) (grid units) and nothing
    elsewhere (the half-open support is the reading that gives exactly w taps
    per dimension, Sec. II-A)."""
    beta = params.kernel_beta(w)
    ns = (20, 15)
    for x, y in [(0.123, -2.9), (-math.pi, 3.1), (1.7, 0.0)]:
        b = direct.spread(([x], [y]), [1.5 - 0.5j], ns, w, beta)
        ref = np.zeros(ns[::-1], dtype=complex)
        g = [(x + math.pi) * ns[0] / (2 * math.pi), (y + math.pi) * ns[1] / (2 * math.pi)]
        for l2 in range(ns[1]):
            for l1 in range(ns[0]):
                wt = 1.0
                for l, gi, n in ((l1, g[0], ns[0]), (l2, g[1], ns[1])):
                    d = (l - gi + n / 2) % n - n / 2
                    wt *= math.exp(beta * (math.sqrt(1 - (2 * d / w) ** 2) - 1)) if -1 <= 2 * d / w < 1 else 0.0
                ref[l2, l1] = wt * (1.5 - 0.5j)
        assert np.allclose(b, ref, atol=1e-14)
        assert np.count_nonzero(b) == w * w


def test_precision_improves_with_eps():
    Ns = (16, 16)
    pts = _pts(400, 2)
    c = _cplx(400)
    ref = direct.type1(pts, c, Ns)
    errs = [nufft.rel_l2(nufft.type1(pts, c, Ns, e), ref) for e in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10)]
    assert all(a > b for a, b in zip(errs, errs[1:]))


# Upsampling sigma < 2 (named as future work in Sec. VI; the width / shape rule
# is the FINUFFT paper's, a reading): pinned only by the exact sums.
SIGMA_CASES = [((16, 12), 1e-3), ((17, 10), 1e-6), ((12, 13), 1e-9), ((8, 10, 6), 1e-5)]


@pytest.mark.parametrize("Ns,eps", SIGMA_CASES)
@pytest.mark.parametrize("sigma", [1.25, 1.5])
def test_upsampling_below_two_matches_direct_sums(Ns, eps, sigma):
    pts = _pts(300, len(Ns))
    c = _cplx(300)
    got = nufft.type1(pts, c, Ns, eps, iflag=-1, sigma=sigma)
    assert nufft.rel_l2(got, direct.type1(pts, c, Ns, iflag=-1)) <= 10 * eps
    f = _cplx(Ns[::-1])
    got = nufft.type2(pts, f, eps, iflag=+1, sigma=sigma)
    assert nufft.rel_l2(got, direct.type2(pts, f, iflag=+1)) <= 10 * eps
    P = nufft.Params(Ns, eps, sigma=sigma)
    assert all(n >= math.ceil(sigma * N) and n < 2 * N + 2 * P.w for n, N in zip(P.ns, Ns))


def test_sigma_two_keeps_the_paper_rule():
    for eps in (1e-2, 1e-5, 1e-9, 1e-12):
        P = nufft.Params((40, 30), eps, sigma=2)
        assert P.w == params.kernel_width(eps) and P.beta == 2.30 * P.w
        assert P.ns == tuple(params.fine_grid_size(N, P.w) for N in (40, 30))
