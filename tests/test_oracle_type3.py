"""Pins for the oracle's 1D sums and its type 3 transform.

1D and type 3 are named in Sec. I-B and Sec. VI as outside the paper's
scope.  The exact type 3 sum is pinned, independently of its summation code,
by the uniform-grid case that reduces to numpy.fft, a one-point closed form
and the shift theorem; the type 3 steps (oracle/nufft.py) are then pinned to
that exact sum within a small multiple of eps, across tolerances, dimensions,
signs and the degenerate cases of the reduction (all points or all
frequencies at one value).
"""
import math

import numpy as np
import pytest

from oracle import direct, nufft, params

R = np.random.default_rng(20210216)


def _cplx(shape):
    return R.standard_normal(shape) + 1j * R.standard_normal(shape)


def _dft_signed(a, iflag):
    if iflag < 0:
        return np.fft.fftn(a)
    return np.fft.ifftn(a) * a.size


# ---------------------------------------------------------------- 1D sums ---

@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("N", [16, 15])
def test_1d_type1_uniform_grid_is_dft(iflag, N):
    x = -math.pi + 2 * math.pi * np.arange(N) / N
    c = _cplx(N)
    f = direct.type1((x,), c, (N,), iflag=iflag)
    # point j sits at 2 pi j / N - pi: the phase exp(-iflag i k pi) = (-1)^k
    k = params.mode_indices(N)
    ref = _dft_signed(c, iflag)[k % N] * np.where(k % 2 == 0, 1.0, -1.0)
    assert np.allclose(f, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("iflag", [-1, 1])
def test_1d_type2_is_adjoint_of_type1(iflag):
    M, N = 300, 37
    x = (R.uniform(-math.pi, math.pi, M),)
    c, f = _cplx(M), _cplx(N)
    a = np.vdot(direct.type1(x, c, (N,), iflag=-iflag), f)
    b = np.vdot(c, direct.type2(x, f, iflag=iflag))
    assert abs(a - b) <= 1e-11 * abs(a)


@pytest.mark.parametrize("eps", [1e-3, 1e-7, 1e-12])
def test_1d_three_step_within_eps(eps):
    M, N = 4000, 200
    x = (R.uniform(-math.pi, math.pi, M),)
    c, f = _cplx(M), _cplx(N)
    e1 = nufft.rel_l2(nufft.type1(x, c, (N,), eps, iflag=1), direct.type1(x, c, (N,), iflag=1))
    e2 = nufft.rel_l2(nufft.type2(x, f, eps, iflag=-1), direct.type2(x, f, iflag=-1))
    assert e1 < 10 * eps and e2 < 10 * eps


# --------------------------------------------------------- exact type 3 ---

@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("Ns", [(12,), (6, 5), (4, 3, 5)])
def test_type3_grid_reduces_to_dft(iflag, Ns):
    """x_j on a tensor grid 2 pi j / n and integer frequencies 0..n-1: the
    type 3 sum is the d-dimensional DFT."""
    dim = len(Ns)
    axes = [2 * math.pi * np.arange(n) / n for n in Ns]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    pts = tuple(m.ravel() for m in mesh[::-1])
    kax = [np.arange(n, dtype=float) for n in Ns]
    kmesh = np.meshgrid(*kax[::-1], indexing="ij")
    freqs = tuple(m.ravel() for m in kmesh[::-1])
    c = _cplx(int(np.prod(Ns)))
    f = direct.type3(pts, c, freqs, iflag=iflag)
    ref = _dft_signed(c.reshape(Ns[::-1]), iflag).ravel()
    assert dim == len(freqs)
    assert np.allclose(f, ref, rtol=0, atol=1e-11)


def test_type3_single_point_closed_form():
    x = (np.array([1.7]), np.array([-2.25]))
    s = (R.uniform(-40, 40, 50), R.uniform(-40, 40, 50))
    f = direct.type3(x, np.array([2.0 - 0.5j]), s, iflag=-1)
    ref = (2.0 - 0.5j) * (np.cos(1.7 * s[0] - 2.25 * s[1]) - 1j * np.sin(1.7 * s[0] - 2.25 * s[1]))
    assert np.allclose(f, ref, rtol=0, atol=1e-13)


def test_type3_shift_theorem():
    """Moving every point by a multiplies f_k by exp(iflag i s_k.a)."""
    M, K = 200, 60
    x = tuple(R.uniform(-3, 3, M) for _ in range(3))
    s = tuple(R.uniform(-10, 10, K) for _ in range(3))
    a = (0.75, -1.5, 2.0)
    c = _cplx(M)
    f0 = direct.type3(x, c, s, iflag=1)
    f1 = direct.type3(tuple(xd + ad for xd, ad in zip(x, a)), c, s, iflag=1)
    ph = np.exp(1j * sum(ad * sd for ad, sd in zip(a, s)))
    assert np.allclose(f1, f0 * ph, rtol=0, atol=1e-10)


def test_type3_subset_matches_full():
    x = tuple(R.uniform(-3, 3, 100) for _ in range(2))
    s = tuple(R.uniform(-8, 8, 40) for _ in range(2))
    c = _cplx(100)
    full = direct.type3(x, c, s)
    idx = np.array([39, 0, 17, 17])
    assert np.array_equal(direct.type3(x, c, s, idx=idx), full[idx])


# ------------------------------------------------------- type 3 steps ---

def _t3_case(dim, M, K, seed, xc=1.3, xw=4.0, sc=-7.0, sw=25.0):
    g = np.random.default_rng(seed)
    x = tuple(g.uniform(xc - xw, xc + xw, M) for _ in range(dim))
    s = tuple(g.uniform(sc - sw, sc + sw, K) for _ in range(dim))
    c = g.standard_normal(M) + 1j * g.standard_normal(M)
    return x, s, c


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("iflag", [-1, 1])
@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-9, 1e-12])
def test_type3_steps_within_eps_of_exact(dim, iflag, eps):
    x, s, c = _t3_case(dim, 1500, 200, seed=dim * 10 + (iflag > 0))
    err = nufft.rel_l2(nufft.type3(x, c, s, eps, iflag=iflag), direct.type3(x, c, s, iflag=iflag))
    assert err < 10 * eps, err


def test_type3_error_decreases_with_eps():
    x, s, c = _t3_case(2, 1500, 200, seed=5)
    ex = direct.type3(x, c, s, iflag=-1)
    errs = [nufft.rel_l2(nufft.type3(x, c, s, e, iflag=-1), ex) for e in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs


@pytest.mark.parametrize("sigma", [1.25, 1.5])
def test_type3_upsampling_below_two(sigma):
    x, s, c = _t3_case(2, 1200, 150, seed=7)
    for eps in (1e-4, 1e-8):
        err = nufft.rel_l2(nufft.type3(x, c, s, eps, iflag=1, sigma=sigma),
                           direct.type3(x, c, s, iflag=1))
        assert err < 10 * eps, (eps, err)


def test_type3_equal_frequencies_in_one_dimension():
    """S = 0 in the second dimension (every frequency has t_k = 3.5)."""
    x, s, c = _t3_case(2, 800, 100, seed=9)
    s = (s[0], np.full(100, 3.5))
    err = nufft.rel_l2(nufft.type3(x, c, s, 1e-9), direct.type3(x, c, s))
    assert err < 1e-8


def test_type3_all_points_equal():
    """X = 0: every point at one place; f is a pure phase times sum c."""
    g = np.random.default_rng(11)
    x = (np.full(50, 0.4), np.full(50, -1.1))
    s = (g.uniform(-30, 30, 80), g.uniform(-30, 30, 80))
    c = g.standard_normal(50) + 1j * g.standard_normal(50)
    err = nufft.rel_l2(nufft.type3(x, c, s, 1e-10), direct.type3(x, c, s))
    assert err < 1e-9


@pytest.mark.parametrize("eps", [1e-3, 1e-12])
def test_type3_taps_stay_inside_grid(eps):
    """Every rescaled point keeps its w taps inside [0, nf) (no wrapping), and
    the rescaled frequencies stay within pi / sigma."""
    for dim in (1, 2, 3):
        x, s, _ = _t3_case(dim, 3000, 500, seed=13 + dim, xw=50.0, sw=3.0)
        w = params.kernel_width(eps)
        for (C, D, gam, h, nf), xd, sd in zip(nufft.type3_params(x, s, w), x, s):
            assert nf % 2 == 0 and params.is_5smooth(nf) and nf >= 2 * w
            g = ((xd - C) / gam + math.pi) / h
            first = np.ceil(g - w / 2)
            assert first.min() >= 0 and (first + w - 1).max() <= nf - 1
            assert np.abs(h * gam * (sd - D)).max() <= math.pi / 2 + 1e-12


def test_1d_spread_interp_are_transposes():
    M, n, w, beta = 500, 64, 7, 16.1
    x = (R.uniform(-math.pi, math.pi, M),)
    c, g = _cplx(M), _cplx(n)
    a = np.vdot(direct.spread(x, c, (n,), w, beta), g)
    b = np.vdot(c, direct.interp(x, g, w, beta))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_1d_single_point_footprint_by_brute_force():
    """One point spreads exp(beta (sqrt(1 - z^2) - 1)), z = 2 (l - g) / w, onto
    exactly the w cells l0 .. l0 + w - 1 with l0 = ceil(g - w/2), wrapped."""
    n, w = 40, 6
    beta = params.kernel_beta(w)
    for xv in (-math.pi, -3.0, 0.1234, 2.9, math.pi - 1e-9):
        grid = direct.spread((np.array([xv]),), np.array([1.0 + 0j]), (n,), w, beta)
        g = (xv + math.pi) * n / (2 * math.pi)
        ref = np.zeros(n)
        for l in range(-n, 2 * n):
            z = 2.0 * (l - g) / w
            if l >= math.ceil(g - w / 2) and l < math.ceil(g - w / 2) + w and abs(z) <= 1:
                ref[l % n] += math.exp(beta * (math.sqrt(1 - z * z) - 1))
        assert np.allclose(grid.real, ref, rtol=0, atol=1e-14) and np.all(grid.imag == 0)
