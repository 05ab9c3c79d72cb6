"""Pins for the oracle's parameter choices and kernel transform (Sec. II)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import params


@pytest.mark.parametrize("eps,w", [
    (1e-2, 3), (1e-3, 4), (1e-4, 5),
    (1e-5, 6),    # Sec. IV-A: eps = 1e-5 gives w = 6
    (1e-6, 7), (1e-7, 8),
    (1e-8, 9),    # Sec. III-A remark: eps < 1e-7 needs w > 8
    (1e-12, 13), (0.5, 2), (0.09, 3),
])
def test_kernel_width(eps, w):
    assert params.kernel_width(eps) == w


def test_kernel_width_clamp_and_args():
    assert params.kernel_width(1e-20) == 16
    assert params.kernel_width(1e-20, wmax=8) == 8
    for bad in (0.0, 1.0, -1e-3, 2.0):
        with pytest.raises(ValueError):
            params.kernel_width(bad)


@pytest.mark.parametrize("N,n", [
    (64, 128), (1024, 2048), (41, 90), (81, 162), (100, 200), (1000, 2000),
    (1024, 2048), (333, 675), (128, 256), (1, 12), (2, 12), (7, 15),
])
def test_fine_grid(N, n):
    # w = 6 (eps 1e-5): n is the smallest 2^q 3^p 5^r >= max(2N, 12)
    assert params.fine_grid_size(N, 6) == n


def test_fine_grid_bruteforce():
    def smooth(v):
        return all(p in (2, 3, 5) for p in _factor(v))

    def _factor(v):
        out, p = [], 2
        while p * p <= v:
            while v % p == 0:
                out.append(p)
                v //= p
            p += 1
        if v > 1:
            out.append(v)
        return out

    for N in range(1, 400):
        for w in (2, 7, 13):
            n = params.fine_grid_size(N, w)
            assert n >= max(2 * N, 2 * w) and smooth(n)
            assert not any(smooth(v) for v in range(max(2 * N, 2 * w), n))


def test_es_kernel_special_values():
    beta = params.kernel_beta(6)
    assert math.isclose(beta, 13.8)
    v = params.es_kernel([0.0, 1.0, -1.0, 1.0000001, -2.0], beta)
    assert v[0] == 1.0
    assert math.isclose(v[1], math.exp(-beta)) and math.isclose(v[2], math.exp(-beta))
    assert v[3] == 0.0 and v[4] == 0.0


@pytest.mark.parametrize("w", [3, 6, 13])
def test_es_fourier_against_qawo(w):
    """The oracle's Gauss-Legendre transform agrees with QUADPACK's
    oscillatory (cosine-weighted) adaptive rule on the untransformed
    integral, a different algorithm."""
    beta = params.kernel_beta(w)

    def phi(z):
        return math.exp(beta * (math.sqrt(max(0.0, 1.0 - z * z)) - 1.0))

    for xi in [0.0, 0.7, 2.0, w * math.pi / 4, w * math.pi / 2, 9.5, 30.0]:
        ref = 2.0 * integrate.quad(phi, 0.0, 1.0, weight="cos", wvar=xi,
                                   epsabs=1e-16, epsrel=1e-14, limit=500)[0]
        got = params.es_fourier(xi, beta)
        assert abs(got - ref) <= 1e-13


def test_mode_indices():
    assert list(params.mode_indices(4)) == [-2, -1, 0, 1]
    assert list(params.mode_indices(5)) == [-2, -1, 0, 1, 2]
    assert list(params.mode_indices(1)) == [0]


def test_correction_factors_shape_and_phase():
    w, beta = 6, params.kernel_beta(6)
    p = params.correction_factors(8, 16, w, beta)
    k = params.mode_indices(8)
    # sign alternates with k (the lattice phase), magnitude is even in k
    assert np.all(np.sign(p) == np.where(k % 2 == 0, 1, -1))
    assert np.allclose(np.abs(p[1:]), np.abs(p[1:][::-1]))
    assert math.isclose(p[4], (2.0 / w) / params.es_fourier(0.0, beta))


def test_density_mtip_values():
    # Table tab:mtip: rho = 1.86 for N = 41, M = 1.02e6 and 3.85 for N = 81, M = 1.64e7
    assert round(params.density(1024 * 1000, [41] * 3), 2) == 1.86
    assert round(params.density(16384 * 1000, [81] * 3), 2) == 3.85


def test_sm_tile_bytes_worked_example():
    # second remark of Sec. III-A: m = (8, 8, 2), w = 8, double complex
    nbytes, eff = params.sm_tile_bytes((8, 8, 2), 8, 16)
    assert nbytes == 40960 and math.isclose(eff, 0.05)


def test_golden_paper_values():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as fh:
        gv = json.load(fh)
    for e in gv["kernel_width"]:
        if "w" in e:
            assert params.kernel_width(e["eps"]) == e["w"]
        else:
            assert params.kernel_width(e["eps"]) > e["w_greater_than"]
    for e in gv["density"]:
        assert round(params.density(e["M"], [e["N"]] * e["dim"]), 2) == e["rho_2dp"]
    for e in gv["sm_tile"]:
        nbytes, eff = params.sm_tile_bytes(e["m"], e["w"], e["bytes_per_cell"])
        assert nbytes == e["bytes"] and math.isclose(eff, e["efficiency"])
