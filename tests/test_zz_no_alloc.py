"""The allocation-free batched density features
(mnufft_density_features_batch_noalloc) against the entry point that takes a
caller-allocated workspace, through the C ABI: two calls in a row, the second
with fewer and smaller point sets, bit for bit; and the size limit."""
import ctypes

import numpy as np
import pytest

import workloads
from paper_2102_08463_amd import lib as L
from tests.gpu_helpers import note

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _sets(counts, kinds, seed):
    import torch
    xs, ys = [], []
    for t, (m, kind) in enumerate(zip(counts, kinds)):
        x, y = workloads.points(kind, m, 2, seed + t)
        xs.append(np.asarray(x, np.float32))
        ys.append(np.asarray(y, np.float32))
    off = np.zeros(len(counts) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return dev(np.concatenate(xs)), dev(np.concatenate(ys)), dev(off)


def _both(T, x, y, off, ldf=262):
    import torch
    lib = L.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = torch.full((T, ldf), -7.0, dtype=torch.float32, device="cuda")
    got = torch.full((T, ldf), -7.0, dtype=torch.float32, device="cuda")
    work = torch.empty((T * L.DENSITY_BATCH_WORK_BYTES // 4,), dtype=torch.int32, device="cuda")
    assert lib.mnufft_density_features_batch(L.F32, T, _vp(off), _vp(x), _vp(y), _vp(ref), ldf,
                                             _vp(work), s) == L.OK
    assert lib.mnufft_density_features_batch_noalloc(L.F32, T, _vp(off), _vp(x), _vp(y), _vp(got),
                                                     ldf, s) == L.OK
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_density_features_match_workspace_version():
    note("noalloc density features: 64 sets then 5 smaller sets")
    rng = np.random.default_rng(11)
    kinds = ["uniform", "cluster", "radial", "gaussian"]
    counts = [int(v) for v in rng.integers(1000, 60000, size=L.DENSITY_NOALLOC_MAX_SETS)]
    x, y, off = _sets(counts, [kinds[t % 4] for t in range(len(counts))], 100)
    ref, got = _both(len(counts), x, y, off)
    assert np.array_equal(ref, got)
    assert np.all(got[:, 256:] == -7.0)   # columns past the 256 features untouched
    # second call: fewer, smaller sets (the shared workspace keeps the first
    # call's partial histograms; none of them may leak into this result)
    counts2 = [37, 0, 500, 4096, 1]
    x2, y2, off2 = _sets(counts2, ["cluster", "uniform", "uniform", "radial", "uniform"], 300)
    ref2, got2 = _both(len(counts2), x2, y2, off2)
    assert np.array_equal(ref2, got2)
    assert np.all(got2[1, :256] == 0.0)   # an empty set has zero features


def test_noalloc_density_features_limit():
    import torch
    note("noalloc density features: size limit")
    lib = L.load()
    T = L.DENSITY_NOALLOC_MAX_SETS + 1
    x = torch.zeros((T,), dtype=torch.float32, device="cuda")
    off = torch.arange(T + 1, dtype=torch.int64, device="cuda")
    feat = torch.empty((T, 256), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.mnufft_density_features_batch_noalloc(L.F32, T, _vp(off), _vp(x), _vp(x), _vp(feat),
                                                     256, s) == L.ERR_ARG
