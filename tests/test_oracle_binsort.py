"""Pins for the oracle's bin keys, bin-sort permutation and subproblems (Sec. III-A)."""
import math

import numpy as np
import pytest

from oracle import binsort

R = np.random.default_rng(11)


def test_keys_of_cell_centres():
    """A point at the centre of cell l (position (l + 1/2) h - pi) lies in bin l // m."""
    n, m = 40, 8
    h = 2 * math.pi / n
    l = np.arange(n)
    x = -math.pi + (l + 0.5) * h
    assert np.array_equal(binsort.bin_keys((x, x), (n, n), (m, m)) % (n // m), l // m)
    # 2D key: x fastest
    y = np.full(n, -math.pi + 17.5 * h)
    assert np.array_equal(binsort.bin_keys((x, y), (n, n), (m, m)), l // m + (n // m) * 2)


def test_keys_periodic_fold():
    n, m = 30, 7   # ragged last bin of width 2
    h = 2 * math.pi / n
    l = np.arange(n)
    x = -math.pi + (l + 0.5) * h
    base = binsort.bin_keys((x, x, x), (n, n, n), (m, m, m))
    for sh in (-2 * math.pi, 2 * math.pi):
        assert np.array_equal(binsort.bin_keys((x + sh, x, x - sh), (n,) * 3, (m,) * 3), base)
    # the edges of the period map to bin 0
    assert binsort.bin_keys(([-math.pi], [math.pi]), (n, n), (m, m))[0] == 0
    assert binsort.grid_coord([math.pi], n)[0] == 0.0
    # non-finite and far-away values are brought into [0, n)
    g = binsort.grid_coord([np.nan, np.inf, 50.0, -77.0], n)
    assert np.all((g >= 0) & (g < n)) and g[0] == 0.0 and g[1] == 0.0


def test_keys_fp32_edge_values():
    """fp32 casts of +-pi lie just outside [-pi, pi) and still fold into range."""
    x = np.array([np.float32(math.pi), np.float32(-math.pi), np.nextafter(np.float32(math.pi), 0)],
                 dtype=np.float32)
    g = binsort.grid_coord(x, 2048)
    assert np.all((g >= 0) & (g < 2048))
    k = binsort.bin_keys((x, x), (2048, 2048), (32, 32))
    # fl32(pi) > pi folds to the first cell; fl32(-pi) < -pi is the last cell
    assert k[0] == 0 and k[1] == 63 + 64 * 63 and k[2] == 63 + 64 * 63


@pytest.mark.parametrize("M", [0, 1, 17, 500])
def test_permutation_bruteforce(M):
    ns, ms = (24, 20), (8, 8)
    pts = tuple(R.uniform(-math.pi, math.pi, M) for _ in range(2))
    keys = binsort.bin_keys(pts, ns, ms)
    t = binsort.permutation(keys)
    ref = sorted(range(M), key=lambda j: (keys[j], j))
    assert list(t) == ref


def test_bin_starts_and_subproblems_bruteforce():
    ns, ms = (32, 32), (8, 8)
    M = 3000
    # heavy clustering: most points in one bin
    x = np.concatenate([R.uniform(-math.pi, math.pi, 500), R.uniform(0, 0.1, M - 500)])
    y = np.concatenate([R.uniform(-math.pi, math.pi, 500), R.uniform(0, 0.1, M - 500)])
    keys = binsort.bin_keys((x, y), ns, ms)
    nb = 16
    st = binsort.bin_starts(keys, nb)
    assert st[0] == 0 and st[-1] == M
    for b in range(nb):
        assert st[b + 1] - st[b] == int(np.sum(keys == b))
    sp = binsort.subproblems(keys, nb, 256)
    assert sp[:, 2].sum() == M and sp[:, 2].max() <= 256
    # consecutive coverage of the sorted order, one bin per subproblem
    pos = 0
    for b, s, L in sp:
        assert s == pos and st[b] <= s and s + L <= st[b + 1]
        pos += L
    # brute force list
    ref = []
    for b in range(nb):
        s = st[b]
        while s < st[b + 1]:
            L = min(256, st[b + 1] - s)
            ref.append((b, s, L))
            s += L
    assert [tuple(r) for r in sp] == ref
