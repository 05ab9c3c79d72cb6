"""Train the parameter selector on the GPU from autotuner timings.

Draws a set of synthetic problems -- 2D: shaped like the batched workload
(modes uniform in {64..512}^2, M lognormal around 2e5 within [1e4, 4e6],
uniform / clustered / radial points); 3D: modes uniform in {32..160}^3, M
lognormal around 1e6 within [3e4, 8e6], uniform / clustered / Gaussian
points -- types 1 and 2, times every autotuner candidate on each with the
library's timer, trains the MLP with the library's kernels and writes the
weights in the library's selector format (mnufft_selector_load) and the
timing table (.npz).

    python -m paper_2102_08463_amd.train_selector --out weights.bin --problems 48
    python -m paper_2102_08463_amd.train_selector --dim 3 --eps 1e-5 --out w3.bin
"""
import argparse
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from paper_2102_08463_amd import lib as L  # noqa: E402
from paper_2102_08463_amd.selector import Selector, targets_from_times  # noqa: E402
from paper_2102_08463_amd.tune import time_candidates  # noqa: E402

KINDS = {2: ("uniform", "cluster", "radial"), 3: ("uniform", "cluster", "gaussian")}


def draw_problems(count, seed, mmax=4_000_000, dim=2):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if dim == 2:
            N = (int(rng.integers(64, 513)), int(rng.integers(64, 513)))
            M = int(np.clip(round(math.exp(math.log(2e5) + rng.standard_normal())), 10_000, mmax))
        else:
            N = tuple(int(rng.integers(32, 161)) for _ in range(3))
            M = int(np.clip(round(math.exp(math.log(1e6) + rng.standard_normal())), 30_000,
                            2 * mmax))
        out.append({"type": 1 + (i % 2), "N": N, "M": M, "kind": KINDS[dim][(i // 2) % 3],
                    "seed": int(seed * 1000 + i)})
    return out


def collect(sel, problems, eps, reps=3, log=print):
    X, T, Mk, raw = [], [], [], []
    for k, p in enumerate(problems):
        pts = [torch.from_numpy(np.asarray(a, dtype=np.float32)).cuda()
               for a in workloads.points(p["kind"], p["M"], len(p["N"]), p["seed"])]
        feat = sel.features(p["type"], p["N"], pts)
        _, ms = time_candidates(p["type"], p["N"], pts, eps, dtype=torch.complex64,
                                candidates=sel.cands, reps=reps)
        t, m = targets_from_times(ms)
        X.append(feat.cpu().numpy())
        T.append(t)
        Mk.append(m)
        raw.append(ms)
        best = int(np.argmin([v if v > 0 else 1e30 for v in ms]))
        log(f"[collect] {k + 1}/{len(problems)} {p} best={sel.names[best]} "
            f"{min(v for v in ms if v > 0):.3f} ms")
    return (np.array(X, np.float32), np.array(T, np.float32), np.array(Mk, np.float32),
            np.array(raw, np.float64))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--table", default=None)
    ap.add_argument("--problems", type=int, default=48)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--margin", type=float, default=0.0,
                    help="predicted log-time margin below which the library asks the autotuner")
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3))
    args = ap.parse_args()
    torch.cuda.set_device(0)
    sel = Selector(args.dim, L.F32, args.eps)
    t0 = time.time()
    probs = draw_problems(args.problems, args.seed, dim=args.dim)
    X, T, Mk, raw = collect(sel, probs, args.eps)
    print(f"[train] collected {len(probs)} problems x {sel.K} candidates in {time.time() - t0:.1f} s",
          flush=True)
    dev = torch.device("cuda:0")
    hist = sel.fit(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev),
                   torch.from_numpy(Mk).to(dev), epochs=args.epochs, log_every=500)
    print(f"[train] loss {hist}", flush=True)
    sel.save(args.out, margin=args.margin)
    if args.table:
        np.savez(args.table, X=X, T=T, mask=Mk, ms=raw, names=np.array(sel.names),
                 problems=np.array([str(p) for p in probs]))


if __name__ == "__main__":
    main()
