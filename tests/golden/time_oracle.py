"""Records the oracle's own timings on this machine, for the CPU baseline.

    PYTHONPATH=. OMP_NUM_THREADS=1 python tests/golden/time_oracle.py [--full] [case ...]

For each full-size case whose stored expected values exist (tests/golden/
<case>.json, written by make_golden.py, which times the full oracle run on one
thread), this script times the oracle on the bounded sample that bench.py
times on the GPU host (the same matrix family at two smaller sizes, one
thread), and writes both into tests/golden/oracle_timing.json.  With --full
the full-size oracle run (analyze + factor, then PCG on the case's seeded
right-hand sides) is timed here as well, right before the sample, so that both
are taken under the same conditions on this machine.  bench.py then
scales the measured full-size time by the ratio of the two hosts' sample
times.  Timings only: no expected value of any test comes from here.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synthetic import laplacian_3d, fv_diffusion_3d, rhs, workload, WORKLOADS  # noqa: E402
from oracle import nd, spand as ospand, pcg as opcg  # noqa: E402

# workload -> (family, generator, sample sides); bench.py's CPU_SAMPLE times the same
SAMPLES = {
    "lap3d_64": ("laplacian_3d", lambda s: laplacian_3d(s), (24, 32)),
    "fv3d_128": ("fv_diffusion_3d(s, 3, 1002)", lambda s: fv_diffusion_3d(s, 3.0, 1002), (24, 32)),
}


def host() -> dict:
    model = platform.processor() or platform.machine()
    with open("/proc/cpuinfo") as f:
        for line in f:
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    return {"model": model, "logical_cpus": os.cpu_count()}


def sample(workload: str, scheme: str, eps: float) -> dict:
    from threadpoolctl import threadpool_limits
    fam, make, sizes = SAMPLES[workload]
    w = WORKLOADS[workload]
    out = {"family": fam, "sizes": list(sizes), "n": [], "factor_s": [], "pcg_iter_s": [],
           "n_cg": []}
    with threadpool_limits(1):
        for s in sizes:
            p = make(s)
            A = p.scipy()
            t0 = time.perf_counter()
            plan = nd.analyze(p.rowptr, p.colind, p.coords, max(0, int(round(np.log2(p.n / 64.0)))),
                              w["skip"])
            F = ospand.factor(A, plan, eps, scheme)
            t1 = time.perf_counter()
            b = rhs(p.n, 1, w["rhs_seed"])[:, 0]
            _, it, _ = opcg.pcg(lambda v: A @ v, lambda v: ospand.apply(F, v), b, w["tol"])
            t2 = time.perf_counter()
            out["n"].append(p.n)
            out["factor_s"].append(t1 - t0)
            out["pcg_iter_s"].append((t2 - t1) / max(it, 1))
            out["n_cg"].append(int(it))
    return out


def full_run(g: dict) -> dict:
    """The oracle on the full-size case, one thread: analyze + factor, PCG."""
    from threadpoolctl import threadpool_limits
    p, w = workload(g["workload"])
    A = p.scipy()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        plan = nd.analyze(p.rowptr, p.colind, p.coords, g["depth"], g["skip"])
        F = ospand.factor(A, plan, g["eps"], g["scheme"])
        t1 = time.perf_counter()
        b = rhs(p.n, g["nrhs"], g["rhs_seed"])
        _, its, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, g["tol"])
        t2 = time.perf_counter()
    return {"factor_s": t1 - t0, "pcg_s": t2 - t1, "n_cg": [int(i) for i in its], "nrhs": g["nrhs"]}


if __name__ == "__main__":
    path = os.path.join(HERE, "oracle_timing.json")
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    args = [a for a in sys.argv[1:] if a != "--full"]
    cases = args or [c for c in ("fv3d_128_SO_1e-2", "lap3d_64_SO_1e-2")]
    for case in cases:
        with open(os.path.join(HERE, case + ".json")) as f:
            g = json.load(f)
        if "--full" in sys.argv:
            full = full_run(g)
            print(case, "full", json.dumps(full), flush=True)
        else:
            full = {"factor_s": g["oracle_seconds"]["factor"], "pcg_s": g["oracle_seconds"]["pcg"],
                    "n_cg": g["n_cg"], "nrhs": g["nrhs"]}
        table[case] = {"host": host(), "full": full,
                       "sample": sample(g["workload"], g["scheme"], g["eps"])}
        print(case, json.dumps(table[case]["sample"]), flush=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
