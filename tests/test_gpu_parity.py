"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bit-exact for the bin-sort permutation, bin starts and subproblem list;
within 10 * eps relative l2 of the exact sums for the transforms; within
rounding of the oracle's spreader / interpolator for the isolated steps.
"""
import math

import numpy as np
import pytest

from oracle import binsort, direct, nufft as onufft
from tests.gpu_helpers import cdtype, make_complex, make_points, note, rel_l2

pytestmark = pytest.mark.gpu


def _plan(*a, **kw):
    from paper_2102_08463_amd import Plan
    return Plan(*a, **kw)


# ---------------------------------------------------------------------------
# bin-sort: bit-exact
SORT_CASES = [
    # (dim, N, M, kind, prec, binsize, msub)
    (2, (64, 64), 100_000, "uniform", "f32", None, 1024),
    (2, (45, 61), 4097, "uniform", "f64", (8, 16), 100),       # odd n, ragged bins and tail
    (2, (64, 64), 30_000, "cluster", "f32", None, 1024),        # heavy bin, many subproblems
    (3, (32, 24, 20), 50_001, "uniform", "f32", None, 512),
    (3, (16, 16, 16), 20_000, "gaussian", "f64", (4, 8, 2), 64),
    (2, (16, 16), 1, "uniform", "f32", None, 1024),
    (2, (300, 200), 70_000, "uniform", "f32", (4, 4), 1024),   # 2 radix passes (>256 bins)
    (3, (128, 128, 128), 300_000, "uniform", "f32", (8, 8, 2), 1024),  # 3 passes (>65536 bins)
]


@pytest.mark.parametrize("case", SORT_CASES, ids=lambda c: f"{c[0]}d-{c[3]}-{c[2]}-{c[4]}")
def test_sort_bit_exact(case):
    import torch
    dim, N, M, kind, prec, binsize, msub = case
    note(f"sort {case}")
    pts64, pts = make_points(kind, M, dim, prec, seed=3)
    p = _plan(1, N, eps=1e-6, dtype=cdtype(prec), binsize=binsize, msub=msub)
    p.setpts(*pts)
    perm, bs = p.get_sort()
    sub, nsub = p.get_subproblems()
    torch.cuda.synchronize()
    inf = p.info()
    ns = inf["nfine"][:dim]
    ms = inf["binsize"][:dim]
    keys = binsort.bin_keys(pts64, ns, ms)
    ref = binsort.permutation(keys)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(bs.cpu().numpy().astype(np.int64), binsort.bin_starts(keys, inf["nbins"]))
    rs = binsort.subproblems(keys, inf["nbins"], msub)
    assert nsub == len(rs)
    assert np.array_equal(sub[:, :3].cpu().numpy().astype(np.int64), rs)
    # repeat: identical result
    p.setpts(*pts)
    perm2, _ = p.get_sort()
    assert torch.equal(perm, perm2)
    p.destroy()


def test_sort_fold_and_edges():
    """Coordinates at +-pi, fp32 casts just outside the period and points in
    [-3pi, 3pi) are binned exactly as the oracle folds them."""
    import torch
    note("sort fold edges")
    R = np.random.default_rng(9)
    base = R.uniform(-math.pi, math.pi, 5000)
    x = np.concatenate([base + 2 * math.pi * R.integers(-1, 2, 5000),
                        [math.pi, -math.pi, 3 * math.pi - 1e-6, -3 * math.pi + 1e-6, 0.0]])
    y = np.concatenate([R.uniform(-math.pi, math.pi, 5000), [0.0, math.pi, -math.pi, 1.0, -1.0]])
    for dt in (np.float32, np.float64):
        xs, ys = x.astype(dt), y.astype(dt)
        p = _plan(1, (40, 30), eps=1e-5, dtype=torch.complex64 if dt == np.float32 else torch.complex128)
        p.setpts(torch.from_numpy(xs).cuda(), torch.from_numpy(ys).cuda())
        perm, bs = p.get_sort()
        inf = p.info()
        keys = binsort.bin_keys((xs.astype(np.float64), ys.astype(np.float64)),
                                inf["nfine"][:2], inf["binsize"][:2])
        assert np.array_equal(perm.cpu().numpy(), binsort.permutation(keys))
        p.destroy()


# ---------------------------------------------------------------------------
# isolated spreading / interpolation against the oracle's plain loops
@pytest.mark.parametrize("method", ["gm", "gmsort", "sm"])
@pytest.mark.parametrize("dim,prec,eps", [(2, "f32", 1e-5), (2, "f64", 1e-12), (3, "f32", 1e-5),
                                          (3, "f64", 1e-9), (2, "f32", 1e-6), (3, "f32", 1e-6)])
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_spread_interp_steps(method, dim, prec, eps, kind):
    import torch
    note(f"spread/interp {method} {dim}d {prec} {eps} {kind}")
    N = (48, 40) if dim == 2 else (20, 24, 18)
    M = 20_000 if dim == 2 else 8_000
    pts64, pts = make_points(kind, M, dim, prec, seed=4)
    c64, c = make_complex(M, prec)
    p = _plan(1, N, eps=eps, dtype=cdtype(prec), method=method, msub=300)
    p.setpts(*pts)
    inf = p.info()
    ns, w, beta = inf["nfine"][:dim], inf["w"], inf["beta"]
    grid = p.spread(c).cpu().numpy()
    ref = direct.spread(pts64, c64, ns, w, beta)
    # GM / GM-sort add single-precision terms with float atomics: a cell that
    # sums K terms is off by about sqrt(K) u, u = 2^-24; uniform points give
    # K ~ rho w^d (tens), clustered ones up to M terms on one cell
    # (sqrt(2e4) u ~ 8.5e-6).  SM adds integers exactly in each tile, so its
    # error is the fixed-point quantum of the tile's bound plus the
    # single-precision evaluation of each term, whatever the clustering.  In
    # single precision with kernels of width 6 or less (eps >= 1e-5) the
    # quantum may be up to 2^-21 of the subproblem's largest strength (terms
    # rounded inside their FMA), a grid error of a few 1e-6 in 3D, which is
    # held to eps / 3 instead.
    if prec == "f32":
        tol = 2e-5 if (kind == "cluster" and method != "sm") else 2e-6
        if method == "sm" and w <= 6:
            tol = max(tol, eps / 3)
    else:
        tol = 1e-12 if (kind == "cluster" and method != "sm") else 1e-13
    assert rel_l2(grid, ref) <= tol
    # interpolation from a random grid
    g64, g = make_complex(tuple(ns[::-1]), prec, seed=5)
    cc = p.interp(g).cpu().numpy()
    refc = direct.interp(pts64, g64, w, beta)
    assert rel_l2(cc, refc) <= tol
    p.destroy()


# ---------------------------------------------------------------------------
# full transforms against the exact sums
def _type1_check(pts64, pts, N, prec, eps, iflag=-1, method="auto", ntr=1, kk=None, **kw):
    dim = len(N)
    M = len(pts64[0])
    c64, c = make_complex((ntr, M) if ntr > 1 else M, prec)
    p = _plan(1, N, ntr, eps, iflag, dtype=cdtype(prec), method=method, **kw)
    p.setpts(*pts)
    f = p.execute(c).cpu().numpy()
    p.destroy()
    c64 = c64.reshape(ntr, M)
    f = f.reshape((ntr,) + tuple(N[::-1]))
    errs = []
    for t in range(ntr):
        if kk is None:
            ref = direct.type1(pts64, c64[t], N, iflag=iflag)
            got = f[t]
        else:
            ref = direct.type1(pts64, c64[t], N, iflag=iflag, kk=kk)
            idx = [np.asarray(k) + n // 2 for k, n in zip(kk, N)]
            got = f[t][np.ix_(*idx[::-1])]
        errs.append(rel_l2(got, ref))
    return max(errs)


def _type2_check(pts64, pts, N, prec, eps, iflag=1, method="auto", ntr=1, idx=None, **kw):
    M = len(pts64[0])
    shape = ((ntr,) if ntr > 1 else ()) + tuple(N[::-1])
    f64, f = make_complex(shape, prec, seed=2)
    p = _plan(2, N, ntr, eps, iflag, dtype=cdtype(prec), method=method, **kw)
    p.setpts(*pts)
    c = p.execute(f).cpu().numpy().reshape(ntr, M)
    p.destroy()
    f64 = f64.reshape((ntr,) + tuple(N[::-1]))
    errs = []
    for t in range(ntr):
        ref = direct.type2(pts64, f64[t], iflag=iflag, idx=idx)
        got = c[t] if idx is None else c[t][idx]
        errs.append(rel_l2(got, ref))
    return max(errs)


def test_config_small_2d_type1():
    """2D type 1, 64x64 modes, M = 1e5 uniform, eps 1e-5, fp32; all modes checked
    against the exact sum, and a separate transform of the first 2000 points."""
    note("2d type1 64x64 M=1e5")
    pts64, pts = make_points("uniform", 100_000, 2, "f32", seed=0)
    assert _type1_check(pts64, pts, (64, 64), "f32", 1e-5) <= 1e-4
    sub64 = tuple(a[:2000] for a in pts64)
    subt = tuple(t[:2000].contiguous() for t in pts)
    assert _type1_check(sub64, subt, (64, 64), "f32", 1e-5) <= 1e-4


EPS_SWEEP = [("f32", e) for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)] + \
            [("f64", e) for e in (1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12)]


@pytest.mark.parametrize("prec,eps", EPS_SWEEP)
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_eps_sweep_2d(prec, eps, kind):
    note(f"eps sweep 2d {prec} {eps} {kind}")
    N = (96, 80)
    pts64, pts = make_points(kind, 30_000, 2, prec, seed=1)
    assert _type1_check(pts64, pts, N, prec, eps) <= 10 * eps
    assert _type2_check(pts64, pts, N, prec, eps) <= 10 * eps


@pytest.mark.parametrize("prec,eps", [("f32", 1e-2), ("f32", 1e-5), ("f64", 1e-9), ("f64", 1e-12)])
@pytest.mark.parametrize("kind", ["uniform", "gaussian"])
def test_eps_sweep_3d(prec, eps, kind):
    note(f"eps sweep 3d {prec} {eps} {kind}")
    N = (24, 20, 16)
    pts64, pts = make_points(kind, 20_000, 3, prec, seed=2)
    assert _type1_check(pts64, pts, N, prec, eps) <= 10 * eps
    assert _type2_check(pts64, pts, N, prec, eps) <= 10 * eps


@pytest.mark.parametrize("method", ["gm", "gmsort", "sm"])
@pytest.mark.parametrize("dim", [2, 3])
def test_methods_and_signs(method, dim):
    note(f"methods {method} {dim}d")
    N = (33, 40) if dim == 2 else (17, 12, 22)
    pts64, pts = make_points("uniform", 12_345, dim, "f32", seed=6)
    for iflag in (-1, 1):
        assert _type1_check(pts64, pts, N, "f32", 1e-5, iflag=iflag, method=method) <= 1e-4
        assert _type2_check(pts64, pts, N, "f32", 1e-5, iflag=iflag, method=method) <= 1e-4


# Grids whose bins, the last one of each dimension included, are at least
# two halos wide: the add-back runs bin by bin (own tile plus a neighbour's
# halo per dimension, periodic), including dimensions of one and two bins,
# narrower last bins (odd n too) and clustered points whose heavy bins hold
# many subproblems (tiles merged in groups first).
TILED_CASES = [
    # (dim, N, binsize, prec, eps, kind, msub)
    (2, (64, 48), (32, 32), "f32", 1e-5, "uniform", 300),
    (2, (64, 48), (32, 32), "f32", 1e-5, "cluster", 300),
    (2, (64, 48), (32, 32), "f32", 1e-5, "cluster", 40),    # bins of > 32 tiles: merged
    (2, (16, 32), (32, 32), "f64", 1e-12, "uniform", 300),  # one bin in x, two in y
    (2, (40, 24), (16, 16), "f64", 1e-9, "cluster", 300),
    (2, (60, 40), (32, 32), "f32", 1e-5, "cluster", 300),   # last bins 24 and 16 wide
    (2, (60, 40), (32, 32), "f64", 1e-12, "uniform", 300),
    (3, (16, 16, 16), (16, 8, 8), "f32", 1e-5, "uniform", 300),
    (3, (16, 16, 16), (16, 8, 8), "f32", 1e-5, "cluster", 300),
    (3, (16, 16, 16), (16, 8, 8), "f64", 1e-5, "cluster", 20),
    (3, (8, 8, 8), (16, 8, 8), "f64", 1e-6, "uniform", 300),    # one bin in x, two in y and z
    (3, (12, 16, 8), (8, 8, 8), "f64", 1e-6, "cluster", 300),
    (3, (20, 12, 14), (16, 8, 8), "f32", 1e-5, "uniform", 300),  # last z bin exactly two halos
    (3, (22, 12, 14), (16, 8, 8), "f64", 1e-5, "cluster", 300),  # n = (45, 24, 30)
]


@pytest.mark.parametrize("case", TILED_CASES,
                         ids=lambda c: f"{c[0]}d-{c[1]}-{c[2]}-{c[3]}-{c[5]}-msub{c[6]}")
def test_spread_binwise_addback(case):
    dim, N, bs, prec, eps, kind, msub = case
    note(f"spread bin-wise add-back {case}")
    M = 20_000 if dim == 2 else 8_000
    pts64, pts = make_points(kind, M, dim, prec, seed=14)
    c64, c = make_complex(M, prec, seed=15)
    p = _plan(1, N, eps=eps, dtype=cdtype(prec), method="sm", binsize=bs, msub=msub)
    p.setpts(*pts)
    inf = p.info()
    ns, w, beta = inf["nfine"][:dim], inf["w"], inf["beta"]
    assert list(inf["binsize"][:dim]) == list(bs)
    if msub < 100:  # some bin holds more than 32 subproblems (tiles merged in groups)
        assert np.bincount(binsort.bin_keys(pts64, ns, bs)).max() > 32 * msub
    P = (w + 1) // 2
    for n, m in zip(ns, bs):
        last = n - (-(-n // m) - 1) * m
        assert min(m, last) >= 2 * P
    grid = p.spread(c).cpu().numpy()
    ref = direct.spread(pts64, c64, ns, w, beta)
    # SM tolerance of test_spread_interp_steps; in single precision the
    # tiles' fixed-point quantum follows the heaviest cell of each tile, so
    # a 3D cluster on a grid this small reaches about 4e-6 (held to eps / 2)
    if prec == "f32":
        tol = max(2e-6, eps / (2 if (dim == 3 and kind == "cluster") else 3)) if w <= 6 else 2e-6
    else:
        tol = 1e-13
    assert rel_l2(grid, ref) <= tol
    f_plan = p.execute(c).cpu().numpy()
    p.destroy()
    # A one-transform batch builds the same subproblems and the same tiles and
    # sums them with the cell-oriented gather: the two type 1 results may
    # differ only by the order of the final additions.
    from paper_2102_08463_amd import Batch
    with Batch(1, [N], [M], eps=eps, dtype=cdtype(prec), binsize=[bs], msub=[msub]) as b:
        b.setpts(*pts)
        f_batch = b.split_modes(b.execute(c))[0].cpu().numpy()
    assert rel_l2(f_plan, f_batch) <= (1e-6 if prec == "f32" else 1e-14)


def test_many_transforms():
    note("ntransf 3")
    pts64, pts = make_points("uniform", 9_999, 2, "f32", seed=8)
    assert _type1_check(pts64, pts, (30, 31), "f32", 1e-6, ntr=3) <= 1e-5
    assert _type2_check(pts64, pts, (30, 31), "f32", 1e-6, ntr=3) <= 1e-5


def test_odd_bins_and_tiny_grids():
    note("tiny grids")
    for N, bs in (((1, 1), None), ((2, 3), None), ((5, 7), (3, 2)), ((64, 64), (64, 64))):
        pts64, pts = make_points("uniform", 777, 2, "f64", seed=10)
        assert _type1_check(pts64, pts, N, "f64", 1e-9, binsize=bs) <= 1e-8
        assert _type2_check(pts64, pts, N, "f64", 1e-9, binsize=bs) <= 1e-8


def test_empty_points():
    import torch
    note("M=0")
    p = _plan(1, (16, 16), eps=1e-5)
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    p.setpts(e, e)
    f = p.execute(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert f.shape == (16, 16) and torch.count_nonzero(f).item() == 0
    p.destroy()
    q = _plan(2, (16, 16), eps=1e-5)
    q.setpts(e, e)
    c = q.execute(torch.ones((16, 16), dtype=torch.complex64, device="cuda"))
    assert c.shape == (0,)
    q.destroy()


@pytest.mark.parametrize("dim,prec", [(2, "f32"), (3, "f64")])
def test_adjoint_identity_gpu(dim, prec):
    """<T1 c, f> = <c, T1^H f> with the adjoint on the same sorted points."""
    import torch
    note(f"adjoint {dim}d {prec}")
    N = (40, 36) if dim == 2 else (16, 18, 12)
    pts64, pts = make_points("uniform", 10_000, dim, prec, seed=12)
    _, c = make_complex(10_000, prec)
    _, f = make_complex(tuple(N[::-1]), prec, seed=13)
    p = _plan(1, N, eps=1e-6 if prec == "f32" else 1e-12, dtype=cdtype(prec))
    p.setpts(*pts)
    lhs = torch.vdot(p.execute(c).flatten(), f.flatten()).item()
    rhs = torch.vdot(c, p.execute_adjoint(f)).item()
    tol = 1e-5 if prec == "f32" else 1e-12
    assert abs(lhs - rhs) <= tol * abs(lhs)
    p.destroy()


def test_validate_pts():
    import torch
    from paper_2102_08463_amd import lib as L
    note("validate_pts")
    p = _plan(1, (16, 16), eps=1e-5, validate_pts=True)
    x = torch.zeros(100, dtype=torch.float32, device="cuda")
    p.setpts(x, x)
    x[7] = float("nan")
    with pytest.raises(L.MnufftError) as ei:
        p.setpts(x, x.clone().zero_())
    assert ei.value.code == L.ERR_PTS
    x[7] = 20.0
    with pytest.raises(L.MnufftError):
        p.setpts(x, x.clone().zero_())
    with pytest.raises(RuntimeError):
        p.execute(torch.zeros(100, dtype=torch.complex64, device="cuda"))
    p.destroy()


def test_default_bins_shrink_to_fit_lds():
    """Wide double-precision kernels: the default 3D bins are halved until the
    padded tiles fit in LDS, so the plan stays on method SM."""
    import torch
    note("default bins shrink (3D fp64 eps 1e-12)")
    p = _plan(1, (24, 20, 16), eps=1e-12, dtype=torch.complex128)
    inf = p.info()
    assert inf["method"] == 3
    assert inf["binsize"][:3] != [16, 8, 8]
    p.destroy()


@pytest.mark.parametrize("ntype", [1, 2])
def test_ewald_slices_fp64_3d(ntype):
    """The application's slice geometry (randomly oriented Ewald caps) in fp64
    at eps 1e-12, against the exact sums."""
    note(f"ewald slices fp64 type {ntype}")
    N = (21, 20, 17)
    pts64, pts = make_points("ewald10", 60 * 10 * 10, 3, "f64", seed=5)
    if ntype == 1:
        assert _type1_check(pts64, pts, N, "f64", 1e-12) <= 1e-11
    else:
        assert _type2_check(pts64, pts, N, "f64", 1e-12) <= 1e-11


@pytest.mark.parametrize("dim,prec,eps", [(2, "f32", 1e-4), (2, "f64", 1e-9), (3, "f32", 1e-4),
                                          (3, "f64", 1e-8)])
@pytest.mark.parametrize("sigma", [1.25, 1.5])
def test_upsampling_below_two(dim, prec, eps, sigma):
    """Upsampling factors below two (smaller fine grids, wider kernels)."""
    note(f"upsampfac {sigma} {dim}d {prec} {eps}")
    N = (45, 38) if dim == 2 else (20, 17, 14)
    pts64, pts = make_points("uniform", 15_000 if dim == 2 else 6_000, dim, prec, seed=9)
    assert _type1_check(pts64, pts, N, prec, eps, upsampfac=sigma) <= 10 * eps
    assert _type2_check(pts64, pts, N, prec, eps, upsampfac=sigma) <= 10 * eps
    p = _plan(1, N, eps=eps, dtype=cdtype(prec), upsampfac=sigma)
    inf = p.info()
    from oracle import params as oparams
    assert inf["upsampfac"] == sigma
    assert inf["nfine"][:dim] == [oparams.fine_grid_size(k, inf["w"], sigma=sigma) for k in N]
    p.destroy()


# ---------------------------------------------------------------------------
# widest kernels: w = 14, 15, 16 (eps 1e-13 .. 1e-15, double precision) in 2D
# and 3D, where the default 3D bins shrink so the padded tiles fit in LDS; the
# error floor there is the rounding of the sums, not eps.
@pytest.mark.parametrize("dim,eps", [(2, 1e-13), (2, 1e-15), (3, 1e-14), (3, 1e-15)])
def test_widest_kernels_fp64(dim, eps):
    note(f"widest kernels {dim}d eps {eps}")
    N = (40, 36) if dim == 2 else (16, 20, 18)
    M = 6_000 if dim == 2 else 3_000
    pts64, pts = make_points("uniform", M, dim, "f64", seed=21)
    p = _plan(1, N, eps=eps, dtype=cdtype("f64"))
    w = p.info()["w"]
    p.destroy()
    assert w == {1e-13: 14, 1e-14: 15, 1e-15: 16}[eps]
    tol = max(10 * eps, 2e-13)
    assert _type1_check(pts64, pts, N, "f64", eps) <= tol
    assert _type2_check(pts64, pts, N, "f64", eps) <= tol


def test_width_clamp_warning():
    """eps beyond the widest kernel: the plan is made at w = 16 (f64) / 8 (f32)
    and the status says the width was capped."""
    import torch
    from paper_2102_08463_amd import lib as L
    note("width clamp")
    p = _plan(1, (32, 32), eps=1e-17, dtype=torch.complex128)
    assert p.status == L.WARN_EPS_CLAMPED and p.info()["w"] == 16
    p.destroy()
    q = _plan(2, (32, 32), eps=1e-9, dtype=torch.complex64)
    assert q.status == L.WARN_EPS_CLAMPED and q.info()["w"] == 8
    q.destroy()


def test_largest_1d_mode_count():
    """N = 2^24, the largest mode count a dimension accepts (fine grid 2^25):
    sampled modes of a type 1 against the exact sum."""
    import torch
    note("1d N=2^24")
    N, M = 1 << 24, 2_000_000
    pts64, pts = make_points("uniform", M, 1, "f32", seed=22)
    c64, c = make_complex(M, "f32", seed=23)
    p = _plan(1, (N,), eps=1e-5, dtype=torch.complex64)
    assert p.info()["nfine"][0] == 1 << 25
    p.setpts(*pts)
    f = p.execute(c).cpu().numpy()
    p.destroy()
    ks = np.sort(np.random.default_rng(24).choice(N, 24, replace=False))
    ks = np.concatenate([ks, [0, N - 1]])
    ex = direct.type1(pts64, c64, (N,), kk=(ks - N // 2,))
    assert rel_l2(f[ks], ex) <= 1e-4


@pytest.mark.parametrize("dim,prec,k", [(2, "f32", -83), (3, "f32", -83), (1, "f32", -83),
                                        (2, "f32", 83), (2, "f64", -660), (2, "f64", 660)])
def test_spread_scale_linear(dim, prec, k):
    """The fixed-point scale of each SM tile follows the tile's own strengths
    (a power of two applied with ldexp), so spreading neither overflows nor
    loses bits for strengths near the bottom or the top of the float range:
    type 1 on 2^k c is 2^k times type 1 on c to rounding (|k| = 83 is about
    1e25 in single precision, 660 about 1e199 in double), and strengths of
    about 1e-25 that are not a power-of-two multiple of the first set (so
    every rounding differs) still meet the tolerance against the exact sums."""
    import torch
    note(f"scale 2^{k} {dim}d {prec}")
    N = {1: (200,), 2: (40, 36), 3: (16, 18, 12)}[dim]
    M = 20_000
    pts64, pts = make_points("cluster", M, dim, prec, seed=31)
    _, c = make_complex(M, prec, seed=32)
    eps = 1e-6 if prec == "f32" else 1e-12
    p = _plan(1, N, eps=eps, dtype=cdtype(prec), method="sm")
    p.setpts(*pts)
    f1 = p.execute(c).cpu().numpy().astype(np.complex128)
    f2 = p.execute(c * 2.0 ** k).cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(f2))
    assert rel_l2(f2 * 2.0 ** -k, f1) <= 1e-12
    if k < 0 and prec == "f32":
        c3 = c * 1e-25
        f3 = p.execute(c3).cpu().numpy()
        ex = direct.type1(pts64, c3.cpu().numpy().astype(np.complex128), N, iflag=-1)
        assert rel_l2(f3, ex) <= 10 * eps
    p.destroy()
