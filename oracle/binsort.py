"""Bin keys, the bin-sort permutation and the subproblem list (Sec. III-A).

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).

A point is inside the bin that holds its integer fine-grid coordinates
l_i = floor((x_i + pi) / h_i); bins are m_1 x m_2 (x m_3) blocks of the fine
grid ordered with the first coordinate fastest.  The permutation t lists the
points of bin 0 first, then bin 1, and so on; within a bin, points keep their
original order (a reading: the paper leaves that order open).  Large bins are
cut into consecutive chunks of at most M_sub points, the subproblems.

The floating-point recipe is fixed so that the result is reproducible bit for
bit: g = fl(fl(x + pi) * S) with S = fl(n / (2 pi)), evaluated in IEEE double
without fused multiply-add; then one periodic correction (add n if g < 0,
then subtract n if g >= n), which is exact for points in [-3 pi, 3 pi).
Anything still outside [0, n) (points beyond three periods, or non-finite
values) is reduced with g - floor(g / n) * n and finally forced into [0, n),
non-finite values mapping to 0.
"""
import numpy as np

PI = np.float64(np.pi)


def grid_coord(x, n):
    """Folded grid coordinate g in [0, n) of coordinates x (any float dtype)."""
    x = np.asarray(x).astype(np.float64)
    S = np.float64(n) / (np.float64(2.0) * PI)
    g = (x + PI) * S
    g = np.where(g < 0.0, g + np.float64(n), g)
    g = np.where(g >= np.float64(n), g - np.float64(n), g)
    bad = ~((g >= 0.0) & (g < np.float64(n)))
    if bad.any():
        with np.errstate(invalid="ignore"):
            gb = g[bad]
            gb = gb - np.floor(gb / np.float64(n)) * np.float64(n)
            gb = np.where(gb >= np.float64(n), gb - np.float64(n), gb)
            gb = np.where((gb >= 0.0) & (gb < np.float64(n)), gb, 0.0)
        g = g.copy()
        g[bad] = gb
    return g


def nbins_per_dim(ns, ms):
    return [-(-int(n) // int(m)) for n, m in zip(ns, ms)]


def bin_keys(pts, ns, ms):
    """Bin index of every point: b_1 + B_1 (b_2 + B_2 b_3), b_i = floor(g_i) // m_i."""
    B = nbins_per_dim(ns, ms)
    key = np.zeros(len(pts[0]), dtype=np.int64)
    stride = 1
    for x, n, m, Bi in zip(pts, ns, ms, B):
        l = np.floor(grid_coord(x, n)).astype(np.int64)
        l = np.where(l >= n, l - n, l)
        key += (l // int(m)) * stride
        stride *= Bi
    return key


def permutation(keys):
    """Stable bin-sort permutation t: sorted position -> original index."""
    return np.argsort(np.asarray(keys), kind="stable").astype(np.int64)


def bin_starts(keys, nbins):
    """Exclusive prefix sums of the per-bin counts, length nbins + 1."""
    counts = np.bincount(np.asarray(keys), minlength=nbins)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def subproblems(keys, nbins, msub):
    """Subproblem list (bin, start, length): each nonempty bin in key order is
    cut into consecutive chunks of at most msub sorted points."""
    starts = bin_starts(keys, nbins)
    out = []
    for b in range(nbins):
        s, e = int(starts[b]), int(starts[b + 1])
        while s < e:
            L = min(msub, e - s)
            out.append((b, s, L))
            s += L
    return np.array(out, dtype=np.int64).reshape(-1, 3)
