"""Shared helpers for the GPU parity tests: seeded inputs on both sides."""
import sys

import numpy as np

import workloads

REAL = {"f32": np.float32, "f64": np.float64}


def note(msg):
    """Name the case about to run on the GPU, flushed, so a crash log shows it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def make_points(kind, M, dim, prec, seed=0):
    """Points as the run precision sees them: (numpy arrays widened to float64,
    torch device tensors of the run precision)."""
    import torch
    pts = workloads.points(kind, M, dim, seed)
    cast = [np.asarray(p, dtype=REAL[prec]) for p in pts]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in cast]
    return tuple(a.astype(np.float64) for a in cast), tuple(dev)


def make_complex(shape, prec, seed=1):
    import torch
    v = workloads.strengths(shape, seed)
    v = v.astype(np.complex64 if prec == "f32" else np.complex128)
    return v.astype(np.complex128), torch.from_numpy(np.ascontiguousarray(v)).cuda()


def make_heavy(shape, prec, seed=1):
    """Heavy-tailed strengths (workloads.heavy_strengths), cast like make_complex."""
    import torch
    v = workloads.heavy_strengths(shape, seed)
    v = v.astype(np.complex64 if prec == "f32" else np.complex128)
    return v.astype(np.complex128), torch.from_numpy(np.ascontiguousarray(v)).cuda()


def cdtype(prec):
    import torch
    return torch.complex64 if prec == "f32" else torch.complex128


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
