"""Pins for the oracle's reference gradients: FP64 central differences of the
exact sums, and the adjoint relations."""
import math

import numpy as np
import pytest

from oracle import direct, grad

R = np.random.default_rng(5)


def _cplx(shape):
    return R.standard_normal(shape) + 1j * R.standard_normal(shape)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("iflag", [-1, 1])
def test_type2_grads_fd(dim, iflag):
    Ns = (6, 5, 4)[:dim]
    M = 12
    pts = tuple(R.uniform(-math.pi, math.pi, M) for _ in range(dim))
    f = _cplx(Ns[::-1])
    g = _cplx(M)

    def loss(p, ff):
        return float(np.real(np.vdot(g, direct.type2(p, ff, iflag=iflag))))

    gf, gx = grad.type2_grads(pts, f, g, iflag=iflag)
    hstep = 1e-6
    for i in range(dim):
        for j in (0, 5, 11):
            pp = [a.copy() for a in pts]
            pm = [a.copy() for a in pts]
            pp[i][j] += hstep
            pm[i][j] -= hstep
            fd = (loss(tuple(pp), f) - loss(tuple(pm), f)) / (2 * hstep)
            assert abs(fd - gx[i][j]) <= 1e-6 * (1 + abs(fd))
    # grad wrt Re f and Im f
    for q in [(0,) * dim, tuple(s - 1 for s in f.shape)]:
        for unit in (1.0, 1j):
            fp = f.copy(); fm = f.copy()
            fp[q] += hstep * unit
            fm[q] -= hstep * unit
            fd = (loss(pts, fp) - loss(pts, fm)) / (2 * hstep)
            ana = gf[q].real if unit == 1.0 else gf[q].imag
            assert abs(fd - ana) <= 1e-6 * (1 + abs(fd))


@pytest.mark.parametrize("iflag", [-1, 1])
def test_type1_grads_fd(iflag):
    Ns = (5, 6)
    M = 10
    pts = tuple(R.uniform(-math.pi, math.pi, M) for _ in range(2))
    c = _cplx(M)
    gfm = _cplx(Ns[::-1])

    def loss(p, cc):
        return float(np.real(np.vdot(gfm, direct.type1(p, cc, Ns, iflag=iflag))))

    gc, gx = grad.type1_grads(pts, c, Ns, gfm, iflag=iflag)
    hstep = 1e-6
    for i in range(2):
        for j in (0, 9):
            pp = [a.copy() for a in pts]
            pm = [a.copy() for a in pts]
            pp[i][j] += hstep
            pm[i][j] -= hstep
            fd = (loss(tuple(pp), c) - loss(tuple(pm), c)) / (2 * hstep)
            assert abs(fd - gx[i][j]) <= 1e-6 * (1 + abs(fd))
    for j in (0, 7):
        for unit in (1.0, 1j):
            cp = c.copy(); cm = c.copy()
            cp[j] += hstep * unit
            cm[j] -= hstep * unit
            fd = (loss(pts, cp) - loss(pts, cm)) / (2 * hstep)
            ana = gc[j].real if unit == 1.0 else gc[j].imag
            assert abs(fd - ana) <= 1e-6 * (1 + abs(fd))
