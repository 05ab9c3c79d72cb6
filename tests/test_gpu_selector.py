"""The selector's hand-written kernels against the oracle: density features
(exact counts), MLP forward / loss gradient / backward / Adam (FP64 numpy),
and the selector's training loop reducing the loss."""
import numpy as np
import pytest

from oracle import binsort, mlp
from tests.gpu_helpers import note, rel_l2

pytestmark = pytest.mark.gpu


def test_density_features_exact():
    import math
    import torch
    from paper_2102_08463_amd.selector import Selector
    from paper_2102_08463_amd import lib as L
    note("density features")
    R = np.random.default_rng(3)
    for M, dt in ((0, np.float32), (1, np.float32), (100_001, np.float32), (50_000, np.float64)):
        x = np.concatenate([R.uniform(-math.pi, math.pi, M // 2), R.normal(0, 0.2, M - M // 2)]).astype(dt)
        y = np.concatenate([R.uniform(-math.pi, math.pi, M // 2), R.normal(1, 0.1, M - M // 2)]).astype(dt)
        if M:
            x[0], y[0] = dt(math.pi), dt(-math.pi)   # edge values fold like the bin-sort
        sel = Selector(2, L.F32 if dt == np.float32 else L.F64, 1e-5)
        f = sel.features(1, (64, 64), [torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()])
        cx = np.floor(binsort.grid_coord(x, 16)).astype(int)
        cy = np.floor(binsort.grid_coord(y, 16)).astype(int)
        cnt = np.bincount(cx + 16 * cy, minlength=256)
        ref = np.log1p(256.0 * cnt / M) if M else np.zeros(256)
        assert np.allclose(f[:256].cpu().numpy(), ref, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("B,K", [(1, 5), (37, 18)])
def test_mlp_kernels_against_oracle(B, K):
    import ctypes
    import torch
    from paper_2102_08463_amd import lib as Lb
    note(f"mlp kernels B={B} K={K}")
    F, H = 262, 64
    lib = Lb.load()
    R = np.random.default_rng(B + K)
    n = lib.mnufft_mlp_nparams(F, H, K)
    assert n == mlp.nparams(F, H, K)
    p = (R.standard_normal(n) * 0.1).astype(np.float32)
    X = R.standard_normal((B, F)).astype(np.float32)
    T = R.standard_normal((B, K)).astype(np.float32)
    mask = (R.uniform(size=(B, K)) > 0.2).astype(np.float32)
    mask[0, 0] = 1
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P, Xd, Td, Md = d(p), d(X), d(T), d(mask)
    H1 = torch.empty((B, H), device="cuda")
    H2 = torch.empty((B, H), device="cuda")
    Y = torch.empty((B, K), device="cuda")
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.mnufft_mlp_forward(F, H, K, vp(P), B, vp(Xd), vp(H1), vp(H2), vp(Y), s) == 0
    h1, h2, y = mlp.forward(p.astype(np.float64), X, F, H, K)
    assert rel_l2(Y.cpu().numpy(), y) <= 1e-5 and rel_l2(H2.cpu().numpy(), h2) <= 1e-5
    dY = torch.empty_like(Y)
    loss = torch.empty((1,), device="cuda")
    assert lib.mnufft_mlp_loss_grad(K, B, vp(Y), vp(Td), vp(Md), vp(dY), vp(loss), s) == 0
    assert abs(loss.item() - mlp.loss(p.astype(np.float64), X, T, mask, F, H, K)) <= 1e-4 * abs(loss.item())
    grads = torch.empty_like(P)
    work = torch.empty((2 * B * H,), device="cuda")
    assert lib.mnufft_mlp_backward(F, H, K, vp(P), B, vp(Xd), vp(H1), vp(H2), vp(dY), vp(work),
                                   vp(grads), s) == 0
    g = mlp.grad(p.astype(np.float64), X, T, mask, F, H, K)
    assert rel_l2(grads.cpu().numpy(), g) <= 1e-4
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    for step in (1, 2):
        assert lib.mnufft_mlp_adam(n, vp(P), vp(grads), vp(m), vp(v), ctypes.c_float(1e-3),
                                   ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-8),
                                   step, s) == 0
    pr, mr, vr = mlp.adam_step(p.astype(np.float64), grads.cpu().numpy().astype(np.float64),
                               np.zeros(n), np.zeros(n), 1)
    pr, mr, vr = mlp.adam_step(pr, grads.cpu().numpy().astype(np.float64), mr, vr, 2)
    assert rel_l2(P.cpu().numpy(), pr) <= 1e-6


def test_training_reduces_loss():
    import torch
    from paper_2102_08463_amd.selector import Selector, F
    from paper_2102_08463_amd import lib as L
    note("selector fit")
    sel = Selector(2, L.F32, 1e-6)
    R = np.random.default_rng(0)
    X = R.standard_normal((64, F)).astype(np.float32)
    Wt = R.standard_normal((F, sel.K)).astype(np.float32) * 0.05
    T = np.abs(X @ Wt).astype(np.float32)
    mask = np.ones_like(T)
    d = lambda a: torch.from_numpy(a).cuda()
    hist = sel.fit(d(X), d(T), d(mask), epochs=600, lr=3e-3, log_every=100)
    assert hist[-1] < 0.2 * hist[0]
