"""Batched transforms of uneven sizes in one launch per stage, against the
exact sums and against one plan per transform."""
import numpy as np
import pytest

import workloads
from oracle import direct
from tests.gpu_helpers import note, rel_l2

pytestmark = pytest.mark.gpu


def _batch_inputs(n_modes, n_points, kinds, prec, seed):
    import torch
    rdt = np.float32 if prec == "f32" else np.float64
    cdt = np.complex64 if prec == "f32" else np.complex128
    pts = []
    for t, (M, kind) in enumerate(zip(n_points, kinds)):
        pts.append([np.asarray(a, dtype=rdt) for a in workloads.points(kind, M, len(n_modes[0]), seed + t)])
    cat = [np.concatenate([p[d] for p in pts]) if pts else np.zeros(0, rdt) for d in range(len(n_modes[0]))]
    tens = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in cat]
    return pts, tens, cdt


@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-11)])
@pytest.mark.parametrize("ntype", [1, 2])
def test_small_mixed_batch(prec, eps, ntype):
    import torch
    from paper_2102_08463_amd import Batch, Plan
    note(f"batch small {prec} {eps} type{ntype}")
    n_modes = [(24, 20), (1, 1), (33, 17), (64, 64), (9, 40)]
    n_points = [5000, 77, 0, 12000, 3001]
    kinds = ["uniform", "uniform", "uniform", "cluster", "uniform"]
    pts, tens, cdt = _batch_inputs(n_modes, n_points, kinds, prec, seed=3)
    rng = np.random.default_rng(5)
    b = Batch(ntype, n_modes, n_points, eps=eps, dtype=torch.complex64 if prec == "f32" else torch.complex128,
              binsize=[(8, 8), (32, 32), (16, 32), (32, 32), (16, 16)], msub=[256, 64, 1024, 500, 2048])
    b.setpts(*tens)
    if ntype == 1:
        cs = [(rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(cdt) for M in n_points]
        out = b.execute(torch.from_numpy(np.concatenate(cs)).cuda())
        fs = b.split_modes(out)
        for t in range(len(n_modes)):
            got = fs[t].cpu().numpy()
            ref = direct.type1(tuple(a.astype(np.float64) for a in pts[t]), cs[t].astype(np.complex128),
                               n_modes[t], iflag=-1)
            if n_points[t] == 0:
                assert np.count_nonzero(got) == 0
            else:
                assert rel_l2(got, ref) <= 10 * eps, t
            # the same transform on its own plan
            if n_points[t]:
                with Plan(1, n_modes[t], 1, eps, -1, dtype=b.dtype, binsize=None) as p:
                    p.setpts(*[torch.from_numpy(a).cuda() for a in pts[t]])
                    single = p.execute(torch.from_numpy(cs[t]).cuda()).cpu().numpy()
                assert rel_l2(got, single) <= 2 * eps
    else:
        fs = [(rng.standard_normal(nm[::-1]) + 1j * rng.standard_normal(nm[::-1])).astype(cdt) for nm in n_modes]
        out = b.execute(torch.from_numpy(np.concatenate([f.ravel() for f in fs])).cuda()).cpu().numpy()
        off = 0
        for t in range(len(n_modes)):
            got = out[off:off + n_points[t]]
            off += n_points[t]
            if n_points[t] == 0:
                continue
            ref = direct.type2(tuple(a.astype(np.float64) for a in pts[t]), fs[t].astype(np.complex128), iflag=+1)
            assert rel_l2(got, ref) <= 10 * eps, t
    b.destroy()


@pytest.mark.parametrize("kind", ["uniform", "cluster", "radial"])
def test_batch_64_fullsize(kind):
    """64 2D transforms, modes uniform in {64..512}^2, M lognormal (median 2e5,
    1e4..4e6), eps 1e-6 fp32, type 1 then type 2; 4 transforms checked at
    sampled modes / points against the exact sums."""
    import torch
    from paper_2102_08463_amd import Batch
    note(f"batch 64 {kind}")
    n_modes, n_points = workloads.batch_descriptors(64)
    kinds = [kind] * 64
    pts, tens, cdt = _batch_inputs(n_modes, n_points, kinds, "f32", seed=100)
    rng = np.random.default_rng(9)
    cs = [(rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(cdt) for M in n_points]
    b1 = Batch(1, n_modes, n_points, eps=1e-6)
    b1.setpts(*tens)
    fs = b1.split_modes(b1.execute(torch.from_numpy(np.concatenate(cs)).cuda()))
    check = [int(i) for i in np.argsort(n_points)[[0, 20, 40, 63]]]
    for t in check:
        kk = tuple(np.sort(rng.choice(np.arange(-(N // 2), N - N // 2), size=24, replace=False)) for N in n_modes[t])
        ref = direct.type1(tuple(a.astype(np.float64) for a in pts[t]), cs[t].astype(np.complex128),
                           n_modes[t], iflag=-1, kk=kk)
        got = fs[t].cpu().numpy()[np.ix_(kk[1] + n_modes[t][1] // 2, kk[0] + n_modes[t][0] // 2)]
        assert rel_l2(got, ref) <= 1e-5, t
    b1.destroy()
    b2 = Batch(2, n_modes, n_points, eps=1e-6)
    b2.setpts(*tens)
    fm = [(rng.standard_normal(nm[::-1]) + 1j * rng.standard_normal(nm[::-1])).astype(cdt) for nm in n_modes]
    c = b2.execute(torch.from_numpy(np.concatenate([f.ravel() for f in fm])).cuda()).cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(n_points)])
    for t in check:
        idx = rng.choice(n_points[t], size=min(500, n_points[t]), replace=False)
        ref = direct.type2(tuple(a.astype(np.float64) for a in pts[t]), fm[t].astype(np.complex128),
                           iflag=+1, idx=idx)
        got = c[offs[t]:offs[t + 1]][idx]
        assert rel_l2(got, ref) <= 1e-5, t
    b2.destroy()


@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-8)])
@pytest.mark.parametrize("ntype", [1, 2])
def test_small_mixed_batch_3d(prec, eps, ntype):
    """3D transforms of different sizes, bins and msub in one batch (four
    classes of equal bins and msub, one transform without points): each
    within 10 eps of its exact sums."""
    import torch
    from paper_2102_08463_amd import Batch
    note(f"batch small 3d {prec} {eps} type{ntype}")
    n_modes = [(12, 10, 14), (20, 16, 8), (9, 9, 9), (16, 16, 16), (6, 20, 10)]
    n_points = [3000, 2500, 0, 4000, 1200]
    kinds = ["uniform", "cluster", "uniform", "gaussian", "uniform"]
    pts, tens, cdt = _batch_inputs(n_modes, n_points, kinds, prec, seed=21)
    rng = np.random.default_rng(6)
    b = Batch(ntype, n_modes, n_points, eps=eps,
              dtype=torch.complex64 if prec == "f32" else torch.complex128,
              binsize=[(8, 8, 8), (16, 8, 4), (8, 8, 8), (16, 8, 8), (16, 8, 4)],
              msub=[256, 1024, 256, 512, 1024])
    b.setpts(*tens)
    if ntype == 1:
        cs = [(rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(cdt) for M in n_points]
        fs = b.split_modes(b.execute(torch.from_numpy(np.concatenate(cs)).cuda()))
        for t in range(len(n_modes)):
            got = fs[t].cpu().numpy()
            if n_points[t] == 0:
                assert np.count_nonzero(got) == 0
                continue
            ref = direct.type1(tuple(a.astype(np.float64) for a in pts[t]),
                               cs[t].astype(np.complex128), n_modes[t], iflag=-1)
            assert rel_l2(got, ref) <= 10 * eps, t
    else:
        fm = [(rng.standard_normal(nm[::-1]) + 1j * rng.standard_normal(nm[::-1])).astype(cdt)
              for nm in n_modes]
        c = b.execute(torch.from_numpy(np.concatenate([f.ravel() for f in fm])).cuda()).cpu().numpy()
        off = 0
        for t in range(len(n_modes)):
            got = c[off:off + n_points[t]]
            off += n_points[t]
            if n_points[t] == 0:
                continue
            ref = direct.type2(tuple(a.astype(np.float64) for a in pts[t]),
                               fm[t].astype(np.complex128), iflag=+1)
            assert rel_l2(got, ref) <= 10 * eps, t
    b.destroy()
