"""Autotuner over the library's candidate parameter sets (mnufft_tune_*).

The timing itself (plan per candidate, HIP-event timed setpts + execute,
median of repeats, early cut of hopeless candidates) runs in the library;
this module allocates the buffers, picks the argmin and keeps a small cache
keyed by problem class.
"""
import ctypes
import json
import math
import os

import torch

from . import lib as L
from .plan import _PREC, _ptr


def problem_class(nufft_type, n_modes, M, eps, dtype, kind=""):
    """Cache key: type, dims, precision, eps, rounded log2 sizes and a tag."""
    lg = lambda v: int(round(math.log2(max(v, 1))))
    return f"t{nufft_type}-d{len(n_modes)}-{'f32' if dtype == torch.complex64 else 'f64'}-" \
           f"e{eps:g}-N{'x'.join(str(lg(n)) for n in n_modes)}-M{lg(M)}-{kind}"


def time_candidates(nufft_type, n_modes, points, eps=1e-6, isign=None, dtype=torch.complex64,
                    candidates=None, reps=3, cutoff=4.0, data=None):
    """Milliseconds of setpts + execute for each candidate (-1: not valid here).
    Returns (candidates, list of ms)."""
    dim = len(n_modes)
    dev = points[0].device
    M = points[0].numel()
    prec = _PREC[dtype]
    if candidates is None:
        candidates = L.tune_candidates(dim, prec, eps)
    isign = isign if isign is not None else (-1 if nufft_type == 1 else 1)
    K = int(torch.tensor(n_modes).prod())
    g = torch.Generator(device="cpu").manual_seed(0)
    c = torch.randn((M,), dtype=dtype, generator=g).to(dev) if data is None or nufft_type == 2 else data
    f = torch.randn((K,), dtype=dtype, generator=g).to(dev) if data is None or nufft_type == 1 else data
    stream = torch.cuda.current_stream(dev).cuda_stream
    arr = (L.Opts * len(candidates))()
    for i, o in enumerate(candidates):
        arr[i] = o
        arr[i].stream = stream
        arr[i].device = dev.index if dev.index is not None else -1
    ms = (ctypes.c_double * len(candidates))()
    nm = (ctypes.c_int64 * 3)(*(list(n_modes) + [1] * (3 - dim)))
    z = points[2] if dim == 3 else None
    L.check(L.load().mnufft_tune_time(nufft_type, dim, nm, isign, float(eps), prec, M,
                                      _ptr(points[0]), _ptr(points[1]), _ptr(z), _ptr(c), _ptr(f),
                                      arr, len(candidates), int(reps), float(cutoff), ms),
            "mnufft_tune_time")
    return candidates, list(ms)


class Autotuner:
    """Exhaustive timing with a JSON cache: {problem class: candidate index}."""

    def __init__(self, cache_path=None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                self.cache = json.load(fh)

    def best(self, nufft_type, n_modes, points, eps=1e-6, dtype=torch.complex64, kind="",
             candidates=None, **kw):
        dim = len(n_modes)
        cands = candidates or L.tune_candidates(dim, _PREC[dtype], eps)
        key = problem_class(nufft_type, n_modes, points[0].numel(), eps, dtype, kind)
        if key in self.cache and self.cache[key] < len(cands):
            return cands[self.cache[key]], None
        cands, ms = time_candidates(nufft_type, n_modes, points, eps, dtype=dtype,
                                    candidates=cands, **kw)
        valid = [(t, i) for i, t in enumerate(ms) if t > 0]
        i = min(valid)[1]
        self.cache[key] = i
        if self.cache_path:
            with open(self.cache_path, "w") as fh:
                json.dump(self.cache, fh, indent=1, sort_keys=True)
        return cands[i], ms
