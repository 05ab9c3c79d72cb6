"""The autotuner: every candidate parameter set it may pick gives a result
within 10 * eps of the exact sums (the choice changes speed, never the
answer beyond rounding), its timings are well formed, and its cache keeps
the choice per problem class."""
import json

import numpy as np
import pytest

from oracle import direct
from tests.gpu_helpers import cdtype, make_complex, make_points, note, rel_l2

pytestmark = pytest.mark.gpu

CASES = [
    # (dim, N, M, kind, ntype, eps)
    (2, (96, 80), 20_000, "uniform", 1, 1e-5),
    (2, (96, 80), 20_000, "cluster", 2, 1e-5),
    (2, (70, 130), 3_001, "radial", 1, 1e-6),
    (3, (24, 20, 16), 30_000, "gaussian", 1, 1e-5),
    (3, (24, 20, 16), 30_000, "uniform", 2, 1e-5),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{c[3]}-t{c[4]}")
def test_every_candidate_matches_direct_sum(case):
    import torch
    from paper_2102_08463_amd import Plan, lib as L
    dim, N, M, kind, ntype, eps = case
    pts64, pts = make_points(kind, M, dim, "f32", seed=11)
    rng = np.random.default_rng(5)
    if ntype == 1:
        c64, c = make_complex(M, "f32", seed=12)
        ref = direct.type1(pts64, c64, N, iflag=-1)
    else:
        f64, f = make_complex(tuple(reversed(N)), "f32", seed=12)
        idx = np.sort(rng.choice(M, size=min(M, 2000), replace=False))
        ref = direct.type2(pts64, f64, iflag=+1, idx=idx)
    for o in L.tune_candidates(dim, L.F32, eps):
        note(f"candidate {L.describe(o)} {case}")
        p = Plan(ntype, N, eps=eps, dtype=torch.complex64, method=int(o.method),
                 binsize=[int(b) for b in o.binsize[:dim]], msub=int(o.msub))
        p.setpts(*pts)
        out = p.execute(c if ntype == 1 else f)
        got = out.cpu().numpy()
        if ntype == 2:
            got = got[idx]
        err = rel_l2(got, ref)
        p.destroy()
        assert err <= 10 * eps, (L.describe(o), err)


def test_timings_and_cache(tmp_path):
    import torch
    from paper_2102_08463_amd import lib as L
    from paper_2102_08463_amd.tune import Autotuner, time_candidates
    note("autotuner timings and cache")
    _, pts = make_points("uniform", 50_000, 2, "f32", seed=2)
    cands, ms = time_candidates(1, (128, 128), pts, 1e-5, reps=2)
    assert len(ms) == len(cands) == len(L.tune_candidates(2, L.F32, 1e-5))
    assert all(t > 0 for t in ms), ms
    path = tmp_path / "tune.json"
    at = Autotuner(str(path))
    best, ms2 = at.best(1, (128, 128), pts, 1e-5, kind="uniform", reps=2)
    assert ms2 is not None
    valid = [t for t in ms2 if t > 0]
    assert L.describe(best) == L.describe(cands[int(np.argmin([t if t > 0 else 1e30 for t in ms2]))])
    assert min(valid) == ms2[[L.describe(c) for c in cands].index(L.describe(best))]
    saved = json.loads(path.read_text())
    assert len(saved) == 1
    # a second tuner reads the cache and times nothing
    again, ms3 = Autotuner(str(path)).best(1, (128, 128), pts, 1e-5, kind="uniform")
    assert ms3 is None and L.describe(again) == L.describe(best)
    torch.cuda.synchronize()
