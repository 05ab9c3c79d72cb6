"""mnufft_execute_sorted: the point-indexed vectors in bin-sorted order.

The result must equal mnufft_execute's after the permutation, bit for bit
for method SM (its spreading sums in exact integer arithmetic and its
interpolation evaluates every point the same way) and to rounding for
GM-sort (floating-point atomics).
"""
import numpy as np
import pytest

from tests.gpu_helpers import cdtype, make_complex, make_points, note

pytestmark = pytest.mark.gpu

CASES = [
    # (modes, precision, eps, M, method, n_trans)
    ((64, 48), "f32", 1e-5, 60_000, "sm", 1),
    ((20, 16, 12), "f64", 1e-10, 20_000, "sm", 2),
    ((700,), "f32", 1e-6, 30_000, "sm", 1),
    ((64, 48), "f64", 1e-9, 20_000, "gmsort", 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{len(c[0])}d-{c[1]}-{c[4]}-t{c[5]}")
def test_sorted_order_matches_execute(case):
    import torch
    from paper_2102_08463_amd import Plan
    N, prec, eps, M, method, ntr = case
    note(f"sorted {case}")
    _, pts = make_points("uniform", M, len(N), prec, seed=71)
    exact = method == "sm"
    for typ in (1, 2):
        p = Plan(typ, N, ntr, eps, dtype=cdtype(prec), method=method)
        p.setpts(*pts)
        perm, _ = p.get_sort()
        perm = perm.long()
        if typ == 1:
            shape = (ntr, M) if ntr > 1 else (M,)
            _, c = make_complex(shape, prec, seed=72)
            ref = p.execute(c)
            got = p.execute_sorted(c[..., perm].contiguous())
        else:
            shape = ((ntr,) if ntr > 1 else ()) + tuple(N[::-1])
            _, f = make_complex(shape, prec, seed=73)
            ref = p.execute(f)[..., perm]
            got = p.execute_sorted(f)
        torch.cuda.synchronize()
        if exact:
            assert torch.equal(got, ref), typ
        else:
            d = (got - ref).abs().max().item() / ref.abs().max().item()
            assert d <= 1e-12, (typ, d)
        p.destroy()


def test_sorted_order_refused_where_undefined():
    import torch
    from paper_2102_08463_amd import Plan, lib as L
    note("sorted refused")
    _, pts = make_points("uniform", 1000, 2, "f32", seed=74)
    p = Plan(1, (16, 16), 1, 1e-5, method="gm")
    p.setpts(*pts)
    lib = L.load()
    assert lib.mnufft_execute_sorted(p._h, None, None) == L.ERR_UNSUPPORTED
    p.destroy()
    q = Plan(3, 2, 1, 1e-5)
    q.setpts(*pts, s=pts[0], t=pts[1])
    assert lib.mnufft_execute_sorted(q._h, None, None) == L.ERR_UNSUPPORTED
    q.destroy()
    torch.cuda.synchronize()
