"""HIP graph capture of mnufft_execute / mnufft_execute_adjoint.

After mnufft_set_stream (which also creates the FFT plan of the second
direction) and one eager call, execution enqueues kernels only, so a caller
can capture it once and replay it.  Each test captures on a side stream,
replays several times with new inputs copied into the captured input buffer,
runs the plan eagerly between replays, and requires every replay to equal
the eager result bit for bit (the SM kernels accumulate in exact integer
arithmetic, so the results do not depend on the order of the atomics).
"""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import cdtype, make_complex, make_points, note

pytestmark = pytest.mark.gpu

CASES = [
    # (type, modes, precision, eps, M)
    (1, (64, 64), "f32", 1e-5, 100_000),
    (2, (64, 64), "f32", 1e-5, 100_000),
    (1, (24, 20, 16), "f64", 1e-9, 30_000),
    (2, (500,), "f32", 1e-6, 50_000),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"type{c[0]}-{len(c[1])}d-{c[2]}")
def test_graph_replays_equal_eager(case):
    import torch
    from paper_2102_08463_amd import Plan
    typ, N, prec, eps, M = case
    note(f"graph {case}")
    _, pts = make_points("uniform", M, len(N), prec, seed=31)
    p = Plan(typ, N, 1, eps, dtype=cdtype(prec))
    p.setpts(*pts)
    shape_in = (M,) if typ == 1 else tuple(N[::-1])
    inputs = [make_complex(shape_in, prec, seed=40 + k)[1] for k in range(4)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    p.set_stream(side)
    with torch.cuda.stream(side):
        # eager references on the plan's stream: forward, and the adjoint of it
        ref_fwd = [p.execute(x) for x in inputs]
        ref_adj = [p.execute_adjoint(y) for y in ref_fwd]
        static_in = inputs[0].clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        static_fwd = p.execute(static_in)
        static_adj = p.execute_adjoint(static_fwd)
    for k in range(len(inputs)):
        static_in.copy_(inputs[k])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(static_fwd, ref_fwd[k]), k
        assert torch.equal(static_adj, ref_adj[k]), k
        # eager work on the same plan between replays
        with torch.cuda.stream(side):
            again = p.execute(inputs[(k + 1) % len(inputs)])
        torch.cuda.synchronize()
        assert torch.equal(again, ref_fwd[(k + 1) % len(inputs)])
    p.destroy()


def test_graph_type3():
    import torch
    from paper_2102_08463_amd import Plan
    note("graph type 3")
    x, s = workloads.type3_sets(20_000, 3_000, 2, seed=5, xc=1.0, xw=4.0, sc=-3.0, sw=40.0)
    xd = [torch.from_numpy(np.asarray(a, np.float32)).cuda() for a in x]
    sd = [torch.from_numpy(np.asarray(a, np.float32)).cuda() for a in s]
    p = Plan(3, 2, 1, 1e-5, -1, dtype=torch.complex64)
    p.setpts(xd[0], xd[1], s=sd[0], t=sd[1])
    inputs = [make_complex(20_000, "f32", seed=50 + k)[1] for k in range(3)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    p.set_stream(side)
    with torch.cuda.stream(side):
        refs = [p.execute(c) for c in inputs]
        static_in = inputs[0].clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        static_out = p.execute(static_in)
    for k in range(len(inputs)):
        static_in.copy_(inputs[k])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(static_out, refs[k]), k
    p.destroy()
