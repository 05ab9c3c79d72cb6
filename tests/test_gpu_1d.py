"""GPU parity of 1D transforms (which the paper leaves out, Sec. I-B): the
same kernels instantiated for one dimension, through the C ABI.

Bit-exact for the bin-sort; within rounding of the oracle for the isolated
spread / interpolation steps; within 10 eps of the exact sums for types 1,
2 and 3; the position gradient against the exact derivative sum; and, at
the benchmark's 1D size, sampled modes and points against exact sums.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import binsort, direct, grad as ograd, nufft as onufft
from tests.gpu_helpers import REAL, cdtype, make_complex, make_points, note, rel_l2

pytestmark = pytest.mark.gpu


def _plan(*a, **kw):
    from paper_2102_08463_amd import Plan
    return Plan(*a, **kw)


SORT_CASES = [
    # (N, M, kind, prec, binsize, msub)
    (1000, 100_000, "uniform", "f32", None, 4096),
    (777, 4097, "uniform", "f64", 100, 64),          # ragged last bin and tail
    (4096, 50_000, "cluster", "f32", 64, 1024),       # heavy bins, many subproblems
    (200_000, 300_000, "uniform", "f32", 64, 1024),   # > 256 bins: two radix passes
]


@pytest.mark.parametrize("case", SORT_CASES, ids=lambda c: f"{c[0]}-{c[2]}-{c[3]}")
def test_1d_sort_bit_exact(case):
    import torch
    N, M, kind, prec, binsize, msub = case
    note(f"1d sort {case}")
    pts64, pts = make_points(kind, M, 1, prec, seed=11)
    p = _plan(1, (N,), eps=1e-6, dtype=cdtype(prec),
              binsize=None if binsize is None else (binsize,), msub=msub)
    p.setpts(*pts)
    perm, bs = p.get_sort()
    sub, nsub = p.get_subproblems()
    torch.cuda.synchronize()
    inf = p.info()
    keys = binsort.bin_keys(pts64, inf["nfine"][:1], inf["binsize"][:1])
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), binsort.permutation(keys))
    assert np.array_equal(bs.cpu().numpy().astype(np.int64), binsort.bin_starts(keys, inf["nbins"]))
    rs = binsort.subproblems(keys, inf["nbins"], msub)
    assert nsub == len(rs)
    assert np.array_equal(sub[:, :3].cpu().numpy().astype(np.int64), rs)
    p.destroy()


@pytest.mark.parametrize("method", ["sm", "gmsort", "gm"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_1d_spread_interp_match_oracle(method, prec):
    note(f"1d spread/interp {method} {prec}")
    N, M = 500, 20_000
    eps = 1e-6 if prec == "f32" else 1e-12
    pts64, pts = make_points("uniform", M, 1, prec, seed=2)
    c64, c = make_complex(M, prec, seed=3)
    p = _plan(1, (N,), eps=eps, dtype=cdtype(prec), method=method)
    p.setpts(*pts)
    inf = p.info()
    grid = p.spread(c).cpu().numpy()
    ref = direct.spread(pts64, c64, inf["nfine"][:1], inf["w"], inf["beta"])
    assert rel_l2(grid, ref) <= (2e-6 if prec == "f32" else 1e-13)
    g64, gd = make_complex(tuple(inf["nfine"][:1]), prec, seed=4)
    cc = p.interp(gd).cpu().numpy()
    refc = direct.interp(pts64, g64, inf["w"], inf["beta"])
    assert rel_l2(cc, refc) <= (2e-6 if prec == "f32" else 1e-13)
    p.destroy()


EPS = [("f32", 1e-2), ("f32", 1e-4), ("f32", 1e-6), ("f64", 1e-8), ("f64", 1e-12)]


@pytest.mark.parametrize("prec,eps", EPS, ids=lambda v: str(v))
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_1d_types_1_2_within_eps(prec, eps, kind):
    note(f"1d type1/2 {prec} {eps} {kind}")
    N, M = 1001, 30_000
    pts64, pts = make_points(kind, M, 1, prec, seed=5)
    c64, c = make_complex(M, prec, seed=6)
    f64, f = make_complex((N,), prec, seed=7)
    p1 = _plan(1, (N,), eps=eps, dtype=cdtype(prec), isign=1)
    p1.setpts(*pts)
    assert rel_l2(p1.execute(c).cpu().numpy(), direct.type1(pts64, c64, (N,), iflag=1)) <= 10 * eps
    p2 = _plan(2, (N,), eps=eps, dtype=cdtype(prec), isign=-1)
    p2.setpts(*pts)
    assert rel_l2(p2.execute(f).cpu().numpy(), direct.type2(pts64, f64, iflag=-1)) <= 10 * eps
    p1.destroy()
    p2.destroy()


def test_1d_adjoint_several_vectors_and_edges():
    import torch
    note("1d adjoint / ntransf / edges")
    N, M = 300, 5_000
    pts64, pts = make_points("uniform", M, 1, "f64", seed=8)
    c64, c = make_complex((2, M), "f64", seed=9)
    f64, f = make_complex((2, N), "f64", seed=10)
    p = _plan(1, (N,), 2, 1e-12, -1, dtype=torch.complex128)
    p.setpts(*pts)
    Ac = p.execute(c).cpu().numpy()
    AHf = p.execute_adjoint(f).cpu().numpy()
    for t in range(2):
        lhs = np.vdot(f64[t], Ac[t])
        rhs = np.vdot(AHf[t], c64[t])
        assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
        assert rel_l2(Ac[t], direct.type1(pts64, c64[t], (N,), iflag=-1)) <= 1e-10
    p.destroy()
    # no points; one mode; odd small N with n = 2w
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    q = _plan(1, (64,), eps=1e-5)
    q.setpts(e)
    out = q.execute(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert out.shape == (64,) and torch.count_nonzero(out).item() == 0
    q.destroy()
    for N in (1, 5):
        pts64, pts = make_points("uniform", 2_000, 1, "f64", seed=N)
        c64, c = make_complex(2_000, "f64", seed=12)
        q = _plan(1, (N,), eps=1e-10, dtype=torch.complex128)
        q.setpts(*pts)
        assert rel_l2(q.execute(c).cpu().numpy(), direct.type1(pts64, c64, (N,))) <= 1e-9
        q.destroy()
    # y given to a 1D plan is refused
    with pytest.raises(ValueError):
        q = _plan(1, (16,), eps=1e-5)
        q.setpts(e, e)


def test_1d_interp_grad():
    import torch
    note("1d interp_grad")
    N, M = 200, 3_000
    pts64, pts = make_points("uniform", M, 1, "f64", seed=13)
    f64, f = make_complex((N,), "f64", seed=14)
    g64, g = make_complex(M, "f64", seed=15)
    p = _plan(2, (N,), eps=1e-12, dtype=torch.complex128, isign=1)
    p.setpts(*pts)
    (gx,) = p.interp_grad(f, g)
    ref = ograd.type2_grad_x(pts64, f64, g64, iflag=1)[0]
    assert rel_l2(gx.cpu().numpy(), ref) <= 1e-9
    p.destroy()


@pytest.mark.parametrize("prec,eps", [("f64", 1e-11), ("f32", 1e-5)])
def test_1d_type3(prec, eps):
    note(f"1d type3 {prec}")
    import torch
    x, s = workloads.type3_sets(20_000, 3_000, 1, seed=16, xc=2.0, xw=30.0, sc=-50.0, sw=80.0)
    xc = np.asarray(x[0], REAL[prec])
    sc = np.asarray(s[0], REAL[prec])
    c64, c = make_complex(20_000, prec, seed=17)
    p = _plan(3, 1, 1, eps, 1, dtype=cdtype(prec))
    p.setpts(torch.from_numpy(xc).cuda(), s=torch.from_numpy(sc).cuda())
    f = p.execute(c).cpu().numpy()
    ex = direct.type3((xc.astype(np.float64),), c64, (sc.astype(np.float64),), iflag=1)
    assert rel_l2(f, ex) <= 10 * eps
    if prec == "f64":
        ref = onufft.type3((xc.astype(np.float64),), c64, (sc.astype(np.float64),), eps, iflag=1)
        assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    p.destroy()


def test_1d_full_size_sampled():
    """The benchmark's 1D workload (N = 2^20 modes, M = 1e7 uniform points,
    eps 1e-5, fp32): sampled modes of type 1 and sampled points of type 2
    against exact sums."""
    import torch
    note("1d full size sampled")
    N, M = 1 << 20, 10_000_000
    pts64, pts = make_points("uniform", M, 1, "f32", seed=0)
    c64, c = make_complex(M, "f32", seed=1)
    f64, f = make_complex((N,), "f32", seed=2)
    p = _plan(1, (N,), eps=1e-5, dtype=torch.complex64)
    p.setpts(*pts)
    out = p.execute(c).cpu().numpy()
    rng = np.random.default_rng(5)
    ks = np.sort(rng.choice(N, 32, replace=False))
    ex = direct.type1(pts64, c64, (N,), kk=(ks - N // 2,))
    assert rel_l2(out[ks], ex) <= 1e-4
    cc = p.execute_adjoint(f).cpu().numpy()
    idx = rng.choice(M, 32, replace=False)
    ex2 = direct.type2(pts64, f64, iflag=1, idx=idx)
    assert rel_l2(cc[idx], ex2) <= 1e-4
    p.destroy()
