"""Learned parameter selector: density features -> MLP -> candidate choice.

Features (F = 262): the library's 16 x 16 point-density histogram
(log(1 + 256 count / M)) and six scalars: log2 M / 24, log2 n_i / 12 for
i = 1..3 (0 if absent), w / 16 and the transform type (0 / 1).  The MLP
(F -> 64 -> 64 -> K, ReLU) predicts for each of the autotuner's K candidates
the log of its run time relative to the fastest one; the selector picks the
argmin.  When the predicted margin to the runner-up is below `margin`, the
choice is flagged uncertain and `Selector.choose` falls back to the
exhaustive autotuner if one is given.  The selector changes only which
parameters run, never the result beyond rounding.

All network arithmetic (forward, loss gradient, backward, Adam) runs in the
library's kernels (mnufft_mlp_*); features come from mnufft_density_features.
"""
import ctypes
import math

import numpy as np
import torch

from . import lib as L
from .plan import _PREC, _ptr

F_HIST = 256
F = F_HIST + 6
H = 64


def _vp(t):
    return _ptr(t)


class Selector:
    def __init__(self, dim, prec, eps, device=None, seed=0):
        self._lib = L.load()
        self.dim, self.prec, self.eps = int(dim), int(prec), float(eps)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.cands = L.tune_candidates(dim, prec, eps)
        self.names = [L.describe(o) for o in self.cands]
        self.K = len(self.cands)
        self.n = int(self._lib.mnufft_mlp_nparams(F, H, self.K))
        g = torch.Generator(device="cpu").manual_seed(seed)
        parts = []
        for fan_in, fan_out in ((F, H), (H, H), (H, self.K)):
            parts.append(torch.randn(fan_in * fan_out, generator=g) * math.sqrt(2.0 / fan_in))
            parts.append(torch.zeros(fan_out))
        self.params = torch.cat(parts).float().to(self.device)
        assert self.params.numel() == self.n
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._work = torch.empty((L.DENSITY_WORK_BYTES // 4,), dtype=torch.int32, device=self.device)
        self._stream = lambda: ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- features ----------------------------------------------------------
    def features(self, nufft_type, n_modes, points):
        """(F,) float32 device tensor for one problem."""
        M = points[0].numel()
        feat = torch.empty((F,), dtype=torch.float32, device=self.device)
        prec = L.F32 if points[0].dtype == torch.float32 else L.F64
        L.check(self._lib.mnufft_density_features(prec, M, _vp(points[0]), _vp(points[1]),
                                                  _vp(feat), _vp(self._work), self._stream()),
                "mnufft_density_features")
        feat[F_HIST:] = torch.tensor(self._scalars(nufft_type, n_modes, M), dtype=torch.float32)
        return feat

    def _scalars(self, nufft_type, n_modes, M):
        w, _, _, _ = L.choose_params(self.eps, self.prec, 1)
        ns = [L.choose_params(self.eps, self.prec, N)[2] for N in n_modes] + [1] * (3 - len(n_modes))
        return [math.log2(max(M, 1)) / 24.0] + [math.log2(n) / 12.0 if n > 1 else 0.0 for n in ns] \
            + [w / 16.0, float(nufft_type - 1)]

    def features_batch(self, nufft_type, n_modes_list, x, y, counts):
        """(T, F) float32 device features of T point sets stored back to back in
        x, y (counts[t] points each): one batched histogram launch pair, one
        host-to-device copy of the scalar features."""
        T = len(counts)
        off = torch.zeros((T + 1,), dtype=torch.int64)
        off[1:] = torch.cumsum(torch.tensor([int(m) for m in counts], dtype=torch.int64), 0)
        off = off.to(self.device)
        feat = torch.empty((T, F), dtype=torch.float32, device=self.device)
        work = torch.empty((T * L.DENSITY_BATCH_WORK_BYTES // 4,), dtype=torch.int32,
                           device=self.device)
        prec = L.F32 if x.dtype == torch.float32 else L.F64
        L.check(self._lib.mnufft_density_features_batch(prec, T, _vp(off), _vp(x), _vp(y),
                                                        _vp(feat), F, _vp(work), self._stream()),
                "mnufft_density_features_batch")
        memo = {}
        scal = []
        for nm, M in zip(n_modes_list, counts):
            key = tuple(nm)
            if key not in memo:
                memo[key] = self._scalars(nufft_type, nm, 1)[1:]
            scal.append([math.log2(max(int(M), 1)) / 24.0] + memo[key])
        feat[:, F_HIST:] = torch.tensor(scal, dtype=torch.float32).to(self.device)
        return feat

    # -- network -----------------------------------------------------------
    def forward(self, X):
        """Predictions (B, K) for features X (B, F); returns (H1, H2, Y)."""
        X = X.contiguous()
        B = X.shape[0]
        H1 = torch.empty((B, H), dtype=torch.float32, device=self.device)
        H2 = torch.empty((B, H), dtype=torch.float32, device=self.device)
        Y = torch.empty((B, self.K), dtype=torch.float32, device=self.device)
        L.check(self._lib.mnufft_mlp_forward(F, H, self.K, _vp(self.params), B, _vp(X), _vp(H1),
                                             _vp(H2), _vp(Y), self._stream()), "mnufft_mlp_forward")
        return H1, H2, Y

    def loss_and_grad(self, X, T, mask):
        """(loss tensor, gradient) of the masked MSE at the current parameters."""
        B = X.shape[0]
        H1, H2, Y = self.forward(X)
        dY = torch.empty_like(Y)
        loss = torch.empty((1,), dtype=torch.float32, device=self.device)
        L.check(self._lib.mnufft_mlp_loss_grad(self.K, B, _vp(Y), _vp(T.contiguous()),
                                               _vp(mask.contiguous()), _vp(dY), _vp(loss),
                                               self._stream()), "mnufft_mlp_loss_grad")
        grads = torch.empty_like(self.params)
        work = torch.empty((2 * B * H,), dtype=torch.float32, device=self.device)
        L.check(self._lib.mnufft_mlp_backward(F, H, self.K, _vp(self.params), B, _vp(X), _vp(H1),
                                              _vp(H2), _vp(dY), _vp(work), _vp(grads),
                                              self._stream()), "mnufft_mlp_backward")
        return loss, grads

    def adam(self, grads, lr=3e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        L.check(self._lib.mnufft_mlp_adam(self.n, _vp(self.params), _vp(grads), _vp(self.m),
                                          _vp(self.v), lr, b1, b2, eps, self.step, self._stream()),
                "mnufft_mlp_adam")

    def fit(self, X, T, mask, epochs=1500, lr=3e-3, log_every=0):
        """Full-batch training; returns the loss every `log_every` epochs (or the last)."""
        hist = []
        for e in range(epochs):
            loss, g = self.loss_and_grad(X, T, mask)
            self.adam(g, lr=lr)
            if log_every and e % log_every == 0:
                hist.append(float(loss.item()))
        hist.append(float(self.loss_and_grad(X, T, mask)[0].item()))
        return hist

    # -- selection ---------------------------------------------------------
    def choose(self, feat, allowed=None, margin=0.05, fallback=None):
        """Index of the predicted fastest candidate among `allowed` (default
        all), its predicted margin to the runner-up, and whether it came from
        the fallback.  `fallback()` (e.g. an exhaustive autotuner) is called
        when the margin is below `margin`."""
        _, _, Y = self.forward(feat.reshape(1, -1))
        y = Y[0].cpu().numpy().astype(np.float64)
        idx = list(range(self.K)) if allowed is None else list(allowed)
        order = sorted(idx, key=lambda i: y[i])
        best = order[0]
        gap = y[order[1]] - y[best] if len(order) > 1 else float("inf")
        if gap < margin and fallback is not None:
            return fallback(), gap, True
        return best, gap, False

    # -- persistence -------------------------------------------------------
    # The library's selector file (mnufft_selector_load): "MNSEL001", int32
    # dim, prec, double eps, int32 F, H, K, double margin, K candidate records
    # of int32 (method, binsize[3], msub), then the float32 parameters.
    MAGIC = b"MNSEL001"

    def save(self, path, margin=0.0):
        head = np.array([self.dim, self.prec], np.int32).tobytes() + \
            np.array([self.eps], np.float64).tobytes() + \
            np.array([F, H, self.K], np.int32).tobytes() + \
            np.array([margin], np.float64).tobytes()
        recs = np.array([[o.method, o.binsize[0], o.binsize[1], o.binsize[2], o.msub]
                         for o in self.cands], np.int32).tobytes()
        with open(path, "wb") as fh:
            fh.write(self.MAGIC + head + recs + self.params.cpu().numpy().astype(np.float32).tobytes())

    @classmethod
    def load(cls, path, device=None):
        raw = open(path, "rb").read()
        if raw[:8] != cls.MAGIC:
            raise ValueError("not a selector file")
        dim, prec = np.frombuffer(raw, np.int32, 2, 8)
        eps = float(np.frombuffer(raw, np.float64, 1, 16)[0])
        f, h, k = np.frombuffer(raw, np.int32, 3, 24)
        s = cls(int(dim), int(prec), eps, device=device)
        if (int(f), int(h), int(k)) != (F, H, s.K):
            raise ValueError("weights were trained for another network or candidate list")
        recs = np.frombuffer(raw, np.int32, 5 * s.K, 44).reshape(s.K, 5)
        mine = [[o.method, o.binsize[0], o.binsize[1], o.binsize[2], o.msub] for o in s.cands]
        if recs.tolist() != mine:
            raise ValueError("weights were trained for another candidate list")
        s.margin = float(np.frombuffer(raw, np.float64, 1, 36)[0])
        s.params = torch.from_numpy(
            np.frombuffer(raw, np.float32, s.n, 44 + 20 * s.K).copy()).float().to(s.device)
        return s


def targets_from_times(ms):
    """(log(t / t_min), mask) for one row of candidate timings (-1 = invalid)."""
    ms = np.asarray(ms, dtype=np.float64)
    ok = ms > 0
    t = np.zeros_like(ms)
    if ok.any():
        t[ok] = np.log(ms[ok] / ms[ok].min())
    return t.astype(np.float32), ok.astype(np.float32)
