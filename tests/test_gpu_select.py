"""Parameter selection through the C ABI: plans with opts.tune (the
autotuner, the learned selector), mnufft_batch_select for a batch, and the
adaptive default bins.  Selection changes which parameters run, never the
result beyond rounding, so every case is also checked against the exact sums.
(The paper chose its bins and subproblem size by hand, Sec. III-A, first
remark.)"""
import os

import numpy as np
import pytest

import workloads
from oracle import direct
from tests.gpu_helpers import make_complex, make_points, note, rel_l2

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2102_08463_amd", "data", "selector_2d_f32_1e-06.bin")
WEIGHTS3 = os.path.join(os.path.dirname(WEIGHTS), "selector_3d_f32_1e-05.bin")


def _check_type1(p, pts64, pts, N, eps, seed=3):
    c64, c = make_complex(len(pts64[0]), "f32", seed=seed)
    p.setpts(*pts)
    f = p.execute(c).cpu().numpy()
    return rel_l2(f, direct.type1(pts64, c64, N, iflag=-1))


@pytest.mark.parametrize("N,dim_bins", [((64, 64), [8, 8]), ((1024, 1024), [32, 32]),
                                        ((512, 128), [16, 16]), ((64, 64, 64), [16, 8, 8]),
                                        ((20, 24, 18), [8, 8, 8])])
def test_default_bins_adaptive(N, dim_bins):
    """Default bins are halved along the longest side, down to 8 cells, while
    the fine grid holds fewer than 1024 bins."""
    import torch
    from paper_2102_08463_amd import Plan
    note(f"default bins {N}")
    p = Plan(1, N, eps=1e-5, dtype=torch.complex64)
    inf = p.info()
    assert inf["binsize"][:len(N)] == dim_bins, (inf["nfine"], inf["binsize"])
    p.destroy()


def test_plan_autotune_through_abi():
    """tune = AUTOTUNE: setpts times the candidates on the points, re-plans
    with the fastest, and the transform stays within 10 eps of the exact sum;
    the choice is the one mnufft_select reports (now cached)."""
    import torch
    from paper_2102_08463_amd import Plan, lib as L
    note("tune autotune plan")
    N, eps = (96, 80), 1e-6
    pts64, pts = make_points("cluster", 30_000, 2, "f32", seed=8)
    p = Plan(1, N, eps=eps, dtype=torch.complex64, tune="autotune")
    e = _check_type1(p, pts64, pts, N, eps)
    assert e <= 10 * eps
    o, src = L.select(1, N, pts, eps, mode="autotune")
    inf = p.info()
    assert src == 1
    assert inf["method"] == o.method and inf["msub"] == o.msub
    assert inf["binsize"][:2] == [min(o.binsize[d], inf["nfine"][d]) for d in range(2)]
    p.destroy()


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
@pytest.mark.parametrize("ntype", [1, 2])
def test_plan_learned_through_abi(ntype):
    """tune = LEARNED with the trained selector registered from its file:
    setpts scores the candidates with the library's network and re-plans with
    the pick; results stay within 10 eps of the exact sums."""
    import torch
    from paper_2102_08463_amd import Plan, lib as L
    note(f"tune learned plan type {ntype}")
    L.selector_load(WEIGHTS)
    N, eps = (200, 150), 1e-6
    pts64, pts = make_points("uniform", 200_000, 2, "f32", seed=9)
    o, src = L.select(ntype, N, pts, eps, mode="learned")
    p = Plan(ntype, N, eps=eps, dtype=torch.complex64, tune="learned")
    p.setpts(*pts)
    inf = p.info()
    assert inf["method"] == o.method and inf["msub"] == o.msub
    if ntype == 1:
        c64, c = make_complex(200_000, "f32", seed=4)
        f = p.execute(c).cpu().numpy()
        assert rel_l2(f, direct.type1(pts64, c64, N, iflag=-1)) <= 10 * eps
    else:
        f64, f = make_complex(N[::-1], "f32", seed=5)
        cj = p.execute(f).cpu().numpy()
        idx = np.random.default_rng(1).choice(200_000, 2000, replace=False)
        assert rel_l2(cj[idx], direct.type2(pts64, f64, iflag=+1, idx=idx)) <= 10 * eps
    print(f"[select] learned pick {L.describe(o)} from source {src}", flush=True)
    p.destroy()
    torch.cuda.synchronize()


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_batch_select_learned():
    """mnufft_batch_select scores every transform of a batch in one pass and
    the batch built with its bins and msub stays within 10 eps of the exact
    sums."""
    import torch
    from paper_2102_08463_amd import Batch, lib as L
    note("batch select learned")
    L.selector_load(WEIGHTS)
    eps = 1e-6
    modes = [(64, 100), (300, 200), (128, 128), (90, 400), (512, 64)]
    npts = [20_000, 5_000, 60_000, 1_000, 30_000]
    kinds = ["uniform", "cluster", "radial", "uniform", "cluster"]
    p64 = [tuple(np.asarray(a, np.float32).astype(np.float64)
                 for a in workloads.points(k, m, 2, 40 + t))
           for t, (k, m) in enumerate(zip(kinds, npts))]
    x = torch.from_numpy(np.concatenate([a[0] for a in p64]).astype(np.float32)).cuda()
    y = torch.from_numpy(np.concatenate([a[1] for a in p64]).astype(np.float32)).cuda()
    bins, msub, src = L.batch_select(1, modes, npts, x, y, eps, mode="learned")
    assert len(bins) == len(modes) and all(m > 0 for m in msub)
    assert all(s in (0, 1) for s in src)
    c64 = [workloads.strengths(m, 60 + t).astype(np.complex64).astype(np.complex128)
           for t, m in enumerate(npts)]
    c = torch.from_numpy(np.concatenate(c64).astype(np.complex64)).cuda()
    b = Batch(1, modes, npts, eps=eps, binsize=bins, msub=msub)
    b.setpts(x, y)
    f = b.execute(c).cpu().numpy()
    off = 0
    for t, (nm, m) in enumerate(zip(modes, npts)):
        k = nm[0] * nm[1]
        ref = direct.type1(p64[t], c64[t], nm, iflag=-1).ravel()
        assert rel_l2(f[off:off + k], ref) <= 10 * eps, t
        off += k
    b.destroy()
    print(f"[select] batch picks {list(zip(bins, msub, src))}", flush=True)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained selector weights")
def test_batch_select_matches_network():
    """The fused selection pass of mnufft_batch_select (histogram counts, then
    one launch for features, network and argmin) picks what the library's
    separate feature and network entry points give, for every transform whose
    two best SM candidates are not within rounding of each other; over calls
    with more, fewer and again more sets (the partial rows it keeps between
    calls must not carry counts over)."""
    import torch
    from paper_2102_08463_amd import lib as L
    from paper_2102_08463_amd.selector import Selector
    note("batch select vs network")
    L.selector_load(WEIGHTS)
    sel = Selector.load(WEIGHTS)
    sm = [k for k, o in enumerate(sel.cands) if o.method == L.METHOD_SM]
    rng = np.random.default_rng(5)
    kinds = ["uniform", "cluster", "radial", "gaussian"]
    for T in (12, 5, 12):
        modes = [(int(rng.integers(32, 400)), int(rng.integers(32, 400))) for _ in range(T)]
        npts = [int(rng.integers(0, 80_000)) if t % 5 else 0 for t in range(T)]
        pts = [workloads.points(kinds[t % 4], m, 2, 70 + t) for t, m in enumerate(npts)]
        x = torch.from_numpy(np.concatenate([np.asarray(p[0], np.float32) for p in pts])).cuda()
        y = torch.from_numpy(np.concatenate([np.asarray(p[1], np.float32) for p in pts])).cuda()
        bins, msub, src = L.batch_select(1, modes, npts, x, y, 1e-6, mode="learned")
        feat = sel.features_batch(1, modes, x, y, npts)
        Y = sel.forward(feat)[2].cpu().numpy()[:, sm]
        checked = 0
        for t in range(T):
            order = np.argsort(Y[t])
            if src[t] != 0 or Y[t][order[1]] - Y[t][order[0]] < 1e-4:
                continue
            o = sel.cands[sm[order[0]]]
            assert bins[t] == tuple(o.binsize[:2]) and msub[t] == o.msub, (T, t)
            checked += 1
        assert checked >= T // 2
        print(f"[select] T={T}: {checked} picks equal the network's", flush=True)


@pytest.mark.skipif(not os.path.exists(WEIGHTS3), reason="no trained 3D selector weights")
def test_plan_learned_3d_through_abi():
    """tune = LEARNED in 3D with the 3D selector: the plan's parameters are
    the network's pick (mnufft_select) and the type 1 result stays within
    10 eps of the exact sums at sampled modes."""
    import torch
    from paper_2102_08463_amd import Plan, lib as L
    note("tune learned plan 3d")
    L.selector_load(WEIGHTS3)
    N, eps, M = (48, 40, 56), 1e-5, 300_000
    pts64, pts = make_points("gaussian", M, 3, "f32", seed=12)
    o, src = L.select(1, N, pts, eps, mode="learned")
    p = Plan(1, N, eps=eps, dtype=torch.complex64, tune="learned")
    c64, c = make_complex(M, "f32", seed=13)
    p.setpts(*pts)
    inf = p.info()
    assert inf["method"] == o.method and inf["msub"] == o.msub
    f = p.execute(c).cpu().numpy()
    rng = np.random.default_rng(3)
    kk = tuple(np.sort(rng.choice(np.arange(-(n // 2), n - n // 2), 6, replace=False)) for n in N)
    ref = direct.type1(pts64, c64, N, iflag=-1, kk=kk)
    got = f[np.ix_(*[k + n // 2 for k, n in zip(kk, N)][::-1])]
    assert rel_l2(got, ref) <= 10 * eps
    print(f"[select] 3D learned pick {L.describe(o)} from source {src}", flush=True)
    p.destroy()
