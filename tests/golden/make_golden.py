"""Writes the stored expected values of the full-size parity tests.

    PYTHONPATH=. python tests/golden/make_golden.py [--jobs J] [name ...]

Every value comes from the FP64 oracle (``oracle/``) on the seeded synthetic
inputs of ``synthetic``; nothing here touches the GPU library.  One JSON file
per case.  A single-matrix case stores, per sparsified step, the (a, k, r, r2)
of every interface in canonical order, nnz(L), the algorithmic flops, and for
the PCG solve the iteration counts, the final relative residuals, the norm of
every solution column and its seeded Gaussian sketch S^T x (256 projections,
``synthetic.sketch``), which a test compares with the GPU solution's sketch to
bound the relative error over all n entries.  It also stores the sketch and
norm of one preconditioner application y = M b (first right-hand side).

The batch case (``batch256``) stores the same per problem of the 256-problem
batch (``synthetic.batch_problems``; depth round(log2(n/64)) each, one right-
hand side with seed 3000 + j), computed problem by problem on J processes.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synthetic import workload, rhs, sketch, batch_problems  # noqa: E402
from oracle import nd, spand as ospand, pcg as opcg  # noqa: E402

# name -> (workload, scheme, eps)
CASES = {
    "lap3d_64_SO_1e-2": ("lap3d_64", "SO", 1e-2),
    "lap3d_64_FO_1e-2": ("lap3d_64", "FO", 1e-2),
    "lap3d_64_SO_1e-1": ("lap3d_64", "SO", 1e-1),
    "lap3d_64_FO_1e-1": ("lap3d_64", "FO", 1e-1),
    "lap3d_64_SO_1e-3": ("lap3d_64", "SO", 1e-3),
    "lap3d_64_FO_1e-3": ("lap3d_64", "FO", 1e-3),
    "fv3d_128_SO_1e-2": ("fv3d_128", "SO", 1e-2),
}
BATCH = "batch256"
SKETCH_SEED = 77        # sketch of the PCG solutions
APPLY_SEED = 78         # sketch of y = M b


def _ranks(F) -> dict:
    steps = {}
    for l, recs in sorted(F.ranks.items()):
        recs = sorted(recs)
        steps[str(l)] = {"p": [int(r[0]) for r in recs], "a": [int(r[1]) for r in recs],
                         "k": [int(r[2]) for r in recs], "r": [int(r[3]) for r in recs],
                         "r2": [int(r[4]) for r in recs]}
    return steps


def _solve(p, depth, skip, eps, scheme, b, tol, with_apply):
    A = p.scipy()
    t0 = time.perf_counter()
    plan = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(A, plan, eps, scheme)
    t1 = time.perf_counter()
    X, its, hists = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
    t2 = time.perf_counter()
    out = {
        "depth": depth, "skip": skip, "eps": eps, "scheme": scheme, "tol": tol,
        "nnz_L": int(F.nnz_L), "flops": float(sum(F.flops.values())),
        "steps": _ranks(F), "n_cg": [int(i) for i in its],
        "relres": [float(h[-1]) for h in hists],
        "x_norm": [float(np.linalg.norm(X[:, j])) for j in range(X.shape[1])],
        "x_sketch": sketch(X, SKETCH_SEED).T.tolist(),     # nrhs x 256
        "oracle_seconds": {"factor": t1 - t0, "pcg": t2 - t1},
    }
    if with_apply:
        y = ospand.apply(F, b[:, 0])
        out["apply_norm"] = float(np.linalg.norm(y))
        out["apply_sketch"] = sketch(y, APPLY_SEED)[:, 0].tolist()
    return out


def make(name: str) -> dict:
    wl, scheme, eps = CASES[name]
    p, w = workload(wl)
    b = rhs(p.n, w["nrhs"], w["rhs_seed"])
    g = _solve(p, w["depth"], w["skip"], eps, scheme, b, w["tol"], True)
    g.update(case=name, workload=wl, nrhs=w["nrhs"], rhs_seed=w["rhs_seed"],
             sketch_seed=SKETCH_SEED, apply_seed=APPLY_SEED)
    return g


def batch_depth(n: int) -> int:
    return max(0, int(round(np.log2(n / 64.0))))


_PROBLEMS = []


def _batch_one(j: int) -> dict:
    from threadpoolctl import threadpool_limits
    if not _PROBLEMS:
        _PROBLEMS.extend(batch_problems())
    p = _PROBLEMS[j]
    with threadpool_limits(1):
        b = rhs(p.n, 1, 3000 + j)
        g = _solve(p, batch_depth(p.n), 4, 1e-2, "SO", b, 1e-10, False)
    g.update(n=p.n, shape=list(p.shape), rhs_seed=3000 + j)
    print(f"batch problem {j}: n={p.n} n_cg={g['n_cg']} {g['oracle_seconds']}", flush=True)
    return g


def make_batch(jobs: int) -> dict:
    sizes = [p.n for p in batch_problems()]
    count = len(sizes)
    # largest first, so that the pool's tail is short
    order = sorted(range(count), key=lambda j: -sizes[j])
    with mp.get_context("spawn").Pool(jobs) as pool:
        res = dict(zip(order, pool.map(_batch_one, order, chunksize=1)))
    return {"case": BATCH, "sketch_seed": SKETCH_SEED, "eps": 1e-2, "scheme": "SO",
            "skip": 4, "tol": 1e-10, "problems": [res[j] for j in range(count)]}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    for name in a.names or [c for c in CASES if not c.startswith("fv3d_128")]:
        g = make_batch(a.jobs) if name == BATCH else make(name)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(g, f, separators=(",", ":"))
        print(name, g.get("n_cg"), g.get("nnz_L"), g.get("oracle_seconds"), flush=True)
