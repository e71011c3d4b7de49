"""Writes the stored expected values of the full-size parity tests.

    PYTHONPATH=. python tests/golden/make_golden.py [name ...]

Every value comes from the FP64 oracle (``oracle/``) on the seeded synthetic
inputs of ``synthetic``; nothing here touches the GPU library.  One JSON file
per case: per sparsified step the (a, k, r, r2) of every interface in canonical
order, nnz(L), the algorithmic flops, and for the PCG solve the iteration count,
the final relative residual and the solution at a seeded sample of indices.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synthetic import workload, rhs  # noqa: E402
from oracle import nd, spand as ospand, pcg as opcg  # noqa: E402

# name -> (workload, scheme, eps)
CASES = {
    "lap3d_64_SO_1e-2": ("lap3d_64", "SO", 1e-2),
    "lap3d_64_FO_1e-2": ("lap3d_64", "FO", 1e-2),
    "lap3d_64_SO_1e-1": ("lap3d_64", "SO", 1e-1),
    "fv3d_128_SO_1e-2": ("fv3d_128", "SO", 1e-2),
}
N_SAMPLE = 64


def make(name: str) -> dict:
    wl, scheme, eps = CASES[name]
    p, w = workload(wl)
    A = p.scipy()
    t0 = time.perf_counter()
    plan = nd.analyze(p.rowptr, p.colind, p.coords, w["depth"], w["skip"])
    F = ospand.factor(A, plan, eps, scheme)
    t1 = time.perf_counter()
    b = rhs(p.n, w["nrhs"], w["rhs_seed"])
    X, its, hists = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, w["tol"])
    t2 = time.perf_counter()
    idx = np.sort(np.random.default_rng(7).choice(p.n, N_SAMPLE, replace=False))
    steps = {}
    for l, recs in sorted(F.ranks.items()):
        recs = sorted(recs)
        steps[str(l)] = {"p": [int(r[0]) for r in recs], "a": [int(r[1]) for r in recs],
                         "k": [int(r[2]) for r in recs], "r": [int(r[3]) for r in recs],
                         "r2": [int(r[4]) for r in recs]}
    return {
        "case": name, "workload": wl, "scheme": scheme, "eps": eps,
        "depth": w["depth"], "skip": w["skip"], "nrhs": w["nrhs"], "rhs_seed": w["rhs_seed"],
        "tol": w["tol"], "nnz_L": int(F.nnz_L), "flops": float(sum(F.flops.values())),
        "steps": steps, "n_cg": [int(i) for i in its],
        "relres": [float(h[-1]) for h in hists],
        "sample_idx": idx.tolist(), "x_sample": X[idx, :].T.tolist(),
        "x_norm": [float(np.linalg.norm(X[:, j])) for j in range(X.shape[1])],
        "oracle_seconds": {"factor": t1 - t0, "pcg": t2 - t1},
    }


if __name__ == "__main__":
    for name in sys.argv[1:] or [c for c in CASES if not c.startswith("fv3d_128")]:
        g = make(name)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(g, f, separators=(",", ":"))
        print(name, g["n_cg"], g["nnz_L"], g["oracle_seconds"], flush=True)
