"""Parity at the full workload sizes, in the launch configuration bench.py
times (default plan options), on outputs the oracle computes one by one:
type 1 on a tensor subset of modes (including the extreme ones), type 2 at
2000 random points, both against the exact sums.

The 2D cases follow the paper's accuracy sweep (Sec. IV: 1024^2 modes,
M = 1e7, eps from 1e-2 to 1e-12, single precision down to 1e-6 and double
below) for uniform and clustered points, plus heavy-tailed strengths whose
magnitudes span about six decades inside every bin.  Each case prints its
measured errors."""
import numpy as np
import pytest

from oracle import direct
from tests.gpu_helpers import cdtype, make_complex, make_heavy, make_points, note, rel_l2

pytestmark = pytest.mark.gpu


def _mode_subset(N, count, rng):
    ks = np.arange(-(N // 2), N - N // 2)
    pick = rng.choice(ks[1:-1], size=count - 2, replace=False)
    return np.sort(np.concatenate([[ks[0], ks[-1]], pick]))


def _run(dim, N, M, kind, prec, eps, ksub, heavy=False):
    from paper_2102_08463_amd import Plan
    rng = np.random.default_rng(2024)
    pts64, pts = make_points(kind, M, dim, prec, seed=0)
    mk = make_heavy if heavy else make_complex
    c64, c = mk(M, prec, seed=1)
    f64, f = mk(tuple(N[::-1]), prec, seed=2)
    p = Plan(1, N, 1, eps, -1, dtype=cdtype(prec))
    p.setpts(*pts)
    fk = p.execute(c).cpu().numpy()
    cj = p.execute_adjoint(f).cpu().numpy()   # type 2 with sign +1
    p.destroy()
    kk = tuple(_mode_subset(n, k, rng) for n, k in zip(N, ksub))
    ref1 = direct.type1(pts64, c64, N, iflag=-1, kk=kk)
    got1 = fk[np.ix_(*[k + n // 2 for k, n in zip(kk, N)][::-1])]
    idx = rng.choice(M, size=2000, replace=False)
    ref2 = direct.type2(pts64, f64, iflag=+1, idx=idx)
    return rel_l2(got1, ref1), rel_l2(cj[idx], ref2)


@pytest.mark.parametrize("kind,prec,eps", [
    ("uniform", "f32", 1e-5), ("cluster", "f32", 1e-5),
    ("uniform", "f32", 1e-6), ("cluster", "f32", 1e-6),
    ("uniform", "f64", 1e-7), ("cluster", "f64", 1e-7),
    ("uniform", "f64", 1e-9), ("cluster", "f64", 1e-9),
    ("uniform", "f64", 1e-12)])
def test_2d_1024_M1e7(kind, prec, eps):
    note(f"fullsize 2d 1024^2 M=1e7 {kind} {prec} {eps}")
    e1, e2 = _run(2, (1024, 1024), 10_000_000, kind, prec, eps, (64, 32))
    print(f"[fullsize] 2d {kind} {prec} eps={eps:g} type1 {e1:.3e} type2 {e2:.3e}")
    assert e1 <= 10 * eps and e2 <= 10 * eps


@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_2d_1024_M1e7_heavy_strengths(kind):
    """Strengths with lognormal magnitudes (six decades between the 0.1% and
    99.9% quantiles) at the tightest single-precision tolerance: the
    fixed-point scale of a tile follows its largest strengths, and the small
    ones must still be resolved to the method's accuracy."""
    note(f"fullsize 2d 1024^2 M=1e7 {kind} heavy-tailed f32 1e-6")
    e1, e2 = _run(2, (1024, 1024), 10_000_000, kind, "f32", 1e-6, (64, 32), heavy=True)
    print(f"[fullsize] 2d {kind} heavy f32 eps=1e-06 type1 {e1:.3e} type2 {e2:.3e}")
    assert e1 <= 1e-5 and e2 <= 1e-5


@pytest.mark.parametrize("kind,eps", [("uniform", 1e-5), ("gaussian", 1e-5), ("uniform", 1e-6)])
def test_3d_128_M2p24(kind, eps):
    note(f"fullsize 3d 128^3 M=2^24 {kind} {eps}")
    e1, e2 = _run(3, (128, 128, 128), 1 << 24, kind, "f32", eps, (16, 16, 8))
    print(f"[fullsize] 3d {kind} f32 eps={eps:g} type1 {e1:.3e} type2 {e2:.3e}")
    assert e1 <= 10 * eps and e2 <= 10 * eps
