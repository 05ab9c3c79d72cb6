"""Seeded synthetic inputs for the NUFFT workloads (shared by tests, bench and smoke).

This module only draws random numbers and lays out point sets; it holds none
of the transform's arithmetic, so both the GPU path and the CPU oracle can be
fed from it without sharing any part of the method.

Point sets (every coordinate in [-pi, pi) before casting):
  uniform          iid uniform on [-pi, pi)^d  ("rand" of Sec. IV)
  cluster          iid uniform on the corner box [0, side)^d  ("cluster" of
                   Sec. IV, which uses side 8h; the default side 2 pi/64 is
                   the clustered 2D workload's square)
  gaussian         iid N(0, sigma^2) per coordinate, wrapped periodically
  radial           spokes through the origin at angles pi s / nspokes, equally
                   spaced radii in (-pi, pi)
  spiral_stack     planes z_p = -pi + 2 pi (p + 1/2)/P, each holding an
                   Archimedean spiral r = pi t, theta = 2 pi turns t, plus
                   N(0, jitter^2) jitter on every coordinate, wrapped
  ewald<S>         (3D) M // S^2 slices of S x S detector points, each a
                   spherical cap through the origin (an Ewald sphere of
                   radius 2 pi seen by a detector of half-width 0.65 pi, all
                   within |q| < pi), turned
                   by an independent uniformly random rotation: the shape of
                   the slicing / merging steps of the paper's application
                   (Sec. V), with no data from it
Type 3 sets (``type3_sets``): points iid uniform on a box of centre xc and
half-width xw per coordinate, frequencies iid uniform on a box of centre sc
and half-width sw (off-centre boxes exercise the shifts of the reduction).
Values: complex with iid N(0, 1) real and imaginary parts.

All draws use numpy's PCG64 generator; results are float64 and the caller
casts to the run precision (the cast values are what both sides see).
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _wrap(a):
    return np.mod(a + math.pi, TWO_PI) - math.pi


def uniform(M, dim, seed=0):
    return tuple(rng(seed).uniform(-math.pi, math.pi, size=(dim, M)))


def cluster(M, dim, seed=0, side=TWO_PI / 64):
    return tuple(rng(seed).uniform(0.0, side, size=(dim, M)))


def gaussian(M, dim, seed=0, sigma=0.1):
    return tuple(_wrap(rng(seed).normal(0.0, sigma, size=(dim, M))))


def radial(M, nspokes=256):
    """nspokes lines through the origin, ceil(M/nspokes) samples each, truncated to M."""
    Q = -(-M // nspokes)
    r = -math.pi + TWO_PI * (np.arange(Q) + 0.5) / Q
    th = math.pi * np.arange(nspokes) / nspokes
    x = np.outer(np.cos(th), r).ravel()[:M]
    y = np.outer(np.sin(th), r).ravel()[:M]
    return (_wrap(x), _wrap(y))


def spiral_stack(M, planes=64, turns=32, jitter=1e-3, seed=0):
    """3D stack of spirals with M // planes samples per plane (M rounded down)."""
    Q = M // planes
    t = (np.arange(Q) + 0.5) / Q
    r = math.pi * t
    th = TWO_PI * turns * t
    zp = -math.pi + TWO_PI * (np.arange(planes) + 0.5) / planes
    x = np.tile(r * np.cos(th), planes)
    y = np.tile(r * np.sin(th), planes)
    z = np.repeat(zp, Q)
    j = rng(seed).normal(0.0, jitter, size=(3, planes * Q))
    return (_wrap(x + j[0]), _wrap(y + j[1]), _wrap(z + j[2]))


def _rotations(n, g):
    """n uniformly random rotation matrices (unit quaternions, Shoemake)."""
    u1, u2, u3 = g.uniform(size=(3, n))
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    w, x = a * np.sin(TWO_PI * u2), a * np.cos(TWO_PI * u2)
    y, z = b * np.sin(TWO_PI * u3), b * np.cos(TWO_PI * u3)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], -2)


def ewald_slices(M, side, seed=0, radius=TWO_PI, half_width=0.65 * math.pi):
    """M // side^2 randomly oriented Ewald-sphere caps of side x side points."""
    ns = M // (side * side)
    t = -half_width + 2 * half_width * (np.arange(side) + 0.5) / side
    u, v = np.meshgrid(t, t, indexing="xy")
    u, v = u.ravel(), v.ravel()
    cap = np.stack([u, v, radius - np.sqrt(radius * radius - u * u - v * v)])  # (3, side^2)
    R = _rotations(ns, rng(seed))                                               # (ns, 3, 3)
    q = np.einsum("sij,jk->isk", R, cap).reshape(3, ns * side * side)
    return tuple(_wrap(q[d]) for d in range(3))


def points(kind, M, dim, seed=0):
    if kind == "uniform":
        return uniform(M, dim, seed)
    if kind == "cluster":
        return cluster(M, dim, seed)
    if kind == "gaussian":
        return gaussian(M, dim, seed)
    if kind == "radial":
        assert dim == 2
        return radial(M)
    if kind == "spiral_stack":
        assert dim == 3
        return spiral_stack(M, seed=seed)
    if kind.startswith("ewald"):
        assert dim == 3
        return ewald_slices(M, int(kind[5:]), seed=seed)
    raise ValueError(kind)


def type3_sets(M, K, dim, seed=0, xc=0.0, xw=math.pi, sc=0.0, sw=512.0):
    """(points, frequencies) of a type 3 problem: d arrays of M and d of K."""
    g = rng(seed)
    x = g.uniform(xc - xw, xc + xw, size=(dim, M))
    s = g.uniform(sc - sw, sc + sw, size=(dim, K))
    return tuple(x), tuple(s)


def strengths(shape, seed=1):
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return re + 1j * im


def heavy_strengths(shape, seed=1, sigma=2.3):
    """Complex strengths with lognormal magnitudes (log-magnitude N(0, sigma^2);
    sigma = 2.3 puts the 0.1% and 99.9% quantiles six decades apart) and
    uniform phases: a wide dynamic range among the points of any one bin."""
    g = rng(seed)
    mag = np.exp(sigma * g.standard_normal(shape))
    ph = g.uniform(0.0, 2.0 * math.pi, size=shape)
    return mag * np.cos(ph) + 1j * (mag * np.sin(ph))


def batch_descriptors(ntransf=64, seed=7, mmin=10_000, mmax=4_000_000, median=200_000):
    """Mode counts and point counts of the batched 2D workload: N_1, N_2 iid
    uniform integers in [64, 512]; M lognormal with the given median, sigma 1,
    clipped to [mmin, mmax]."""
    g = rng(seed)
    N = g.integers(64, 513, size=(ntransf, 2))
    M = np.clip(np.round(np.exp(math.log(median) + g.standard_normal(ntransf))), mmin, mmax)
    return [(int(a), int(b)) for a, b in N], [int(m) for m in M]
