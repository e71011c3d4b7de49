"""Benchmark of the spaND hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--eps 1e-2] [--scheme SO]
                    [--no-cpu-baseline]
                    [--workload fv3d_128|lap3d_64|lap2d_64|c1grid|batch256|serve|eig2d|table1]

Default workload: the largest single matrix of the metric's configurations,
3D finite-volume diffusion on a 128^3 grid (n = 2,097,152) with per-cell
coefficient 10^u, u ~ U[-3,3] (seed 1002), harmonic-mean faces, nested-
dissection depth 15, skip 4, eps 1e-2, full second-order scheme, FP64, one
right-hand side ~ N(0,1) (seed 2002), PCG to 1e-10 relative residual.
`--workload lap3d_64` runs the 3D 7-point Laplacian 64^3 (depth 12, 4 RHS);
`c1grid` runs it over eps in {1e-1, 1e-2, 1e-3} x {first, second order}.
Synthetic inputs (synthetic.workload).

One step = the numeric hot path on the device: spand_factor (leaf assembly,
interior elimination, scaling, sparsification, merge, per level) followed by
spand_pcg on the right-hand sides (apply + SpMV + BLAS-1 per iteration).
The symbolic analysis (host C++) depends only on the sparsity pattern and the
coordinates; it is computed once and reported separately (analyze_s).

Prints one JSON line: solves/s (right-hand sides brought to 1e-10 per second,
factorization included), factor TFLOP/s, the p50/p99 of the per-step solve
latency, the roofline of the dominant kernel (live HIP-event timing inside the
library) and the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector / matrix, dense
WORKLOAD_NAMES = {
    "lap3d_64": "lap3d 64^3 7-point Laplacian",
    "lap2d_64": "lap2d 64^2 5-point Laplacian",
    "fv3d_128": "fv3d 128^3 finite-volume diffusion, k = 10^U[-3,3] per cell",
}
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
# dense matrix-core peaks of the GEMM's arithmetic per precision option
# (FP32_BF16: the Schur products on BF16 MFMA; the other GEMMs stay FP32)
PEAK_GEMM_TFLOPS = {"FP64": 78.6, "FP32": 157.3, "FP32_BF16": 157.3}
# kernels whose recorded work is flops (the others record bytes moved)
FLOP_KERNELS = ("k_gemm", "k_gemm_small", "k_potrf_inv", "k_cpqr", "k_cpqr_coop")
# arithmetic of the factorization per precision option (PCG is FP64 always)
DTYPES = {"FP64": "f64", "FP32": "f32 factor, f64 PCG", "FP32_BF16": "f32 factor, bf16 Schur, f64 PCG"}


def kernel_work(breakdown: dict, per: int, precision: str) -> dict:
    """Per-kernel algorithmic work and rate of one step, for the kernels whose
    launches record it: flops (GEMM 2mnk per term, Cholesky n^3/3 per block,
    pivoted QR 4(a-j)(k-j) per reflector) or HBM bytes (copy, fill, scatter)."""
    out = {}
    for k, (ms, calls, work) in sorted(breakdown.items(), key=lambda kv: -kv[1][0]):
        if work <= 0 or ms <= 0:
            continue
        e = {"ms": round(ms / per, 3), "calls": int(calls // per)}
        if k in FLOP_KERNELS:
            tf = work / (ms * 1e-3) / 1e12
            peak = PEAK_GEMM_TFLOPS[precision] if k.startswith("k_gemm") else PEAK_FP64_TFLOPS
            e.update({"gflop": round(work / per / 1e9, 3), "tflops": round(tf, 3),
                      "frac_peak": round(tf / peak, 4), "peak_tflops": peak})
        else:
            gbs = work / (ms * 1e-3) / 1e9
            e.update({"gbytes": round(work / per / 1e9, 3), "gbs": round(gbs, 1),
                      "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)})
        out[k] = e
    return out


# oracle sample of each single-matrix workload: the same matrix family at two
# smaller sizes (seconds each)
CPU_SAMPLE = {
    "lap3d_64": ("laplacian_3d", lambda s: __import__("synthetic").laplacian_3d(s), (24, 32)),
    "fv3d_128": ("fv_diffusion_3d(s, 3, 1002)",
                 lambda s: __import__("synthetic").fv_diffusion_3d(s, 3.0, 1002), (24, 32)),
    "lap2d_64": ("laplacian_2d", lambda s: __import__("synthetic").laplacian_2d(s), (32, 48)),
}


def host_cpu() -> dict:
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def time_oracle(prob, depth, skip, scheme, eps, tol, rhs_seed):
    """(analyze + factor seconds, PCG seconds per iteration, iterations) of the
    oracle on one problem and one right-hand side."""
    from synthetic import rhs
    from oracle import nd, spand as ospand, pcg as opcg
    A = prob.scipy()
    t0 = time.perf_counter()
    plan = nd.analyze(prob.rowptr, prob.colind, prob.coords, depth, skip)
    F = ospand.factor(A, plan, eps, scheme)
    t1 = time.perf_counter()
    b = rhs(prob.n, 1, rhs_seed)[:, 0]
    _, it, _ = opcg.pcg(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
    t2 = time.perf_counter()
    return t1 - t0, (t2 - t1) / max(it, 1), it


def oracle_sample(workload: str, w: dict, scheme: str, eps: float, threads: int = 1,
                  sizes=None) -> dict:
    """The oracle timed on the sample sizes of a workload (analyze + factor,
    PCG per iteration), on `threads` BLAS threads."""
    from threadpoolctl import threadpool_limits
    fam, make, default_sizes = CPU_SAMPLE[workload]
    sizes = list(sizes or default_sizes)
    out = {"family": fam, "sizes": sizes, "n": [], "factor_s": [], "pcg_iter_s": [], "n_cg": [],
           "threads": threads}
    with threadpool_limits(threads):
        for s_ in sizes:
            p = make(s_)
            tf, ti, it = time_oracle(p, max(0, int(round(np.log2(p.n / 64.0)))), w["skip"],
                                     scheme, eps, w["tol"], w["rhs_seed"])
            out["n"].append(p.n)
            out["factor_s"].append(tf)
            out["pcg_iter_s"].append(ti)
            out["n_cg"].append(it)
    return out


def cpu_baseline(workload: str, w: dict, n_full: int, scheme: str, eps: float, n_cg: list) -> dict:
    """The oracle (Python/NumPy FP64) as the CPU baseline of a workload.

    The full-size oracle run is too long to repeat here (about an hour at
    128^3), so this host times a bounded sample instead: the same matrix
    family at two smaller sizes, on one thread (the paper's protocol).  When
    the full-size oracle run was timed on the machine that wrote the stored
    expected values (tests/golden/oracle_timing.json, which holds that run and
    the same sample timed there), the baseline is that measured full-size time
    scaled by the ratio of this host's sample time to that machine's.  A power
    law per phase fitted through the two sample sizes is reported beside it,
    with its prediction for the measured full run, so the error of a pure
    size extrapolation stays visible (without stored timings the power law is
    the baseline).  All host threads are timed on the smaller sample size, and
    their speed-up over one thread is applied to the same estimate."""
    one = oracle_sample(workload, w, scheme, eps, 1)
    ns, tf, ti = one["n"], one["factor_s"], one["pcg_iter_s"]
    nrhs = w["nrhs"]

    def law(t):
        p = np.log(t[1] / t[0]) / np.log(ns[1] / ns[0])
        return (lambda n: t[0] * (n / ns[0]) ** p), float(p)

    ff, pf = law(tf)
    fi, pi = law(ti)
    iters = float(np.sum(n_cg))
    t_law = ff(n_full) + fi(n_full) * iters
    case = f"{workload}_{scheme}_{eps:.0e}".replace("e-0", "e-")
    stored = None
    tpath = os.path.join(ROOT, "tests", "golden", "oracle_timing.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            stored = json.load(f).get(case)
    out = {"unit": "solves/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
           "sample_s": {k: one[k] for k in ("sizes", "n", "factor_s", "pcg_iter_s", "n_cg")}}
    law_txt = (f"power law through the sample (factor exponent {pf:.2f}, PCG per-iteration exponent "
               f"{pi:.2f})")
    if stored and stored["sample"]["sizes"] == one["sizes"]:
        sref = stored["sample"]
        speed = (sum(tf) + sum(ti)) / (sum(sref["factor_s"]) + sum(sref["pcg_iter_s"]))
        full = stored["full"]
        # the stored run's PCG time per iteration, at this run's iteration counts
        t_est = speed * (full["factor_s"] + full["pcg_s"] / max(1, sum(full["n_cg"])) * iters)
        t_law_stored = ff(n_full) + fi(n_full) * float(sum(full["n_cg"]))
        out.update(value=nrhs / t_est, predicted_s_per_step=t_est, sample=(
            f"oracle full run of this workload ({case}: factor {full['factor_s']:.0f} s, PCG "
            f"{full['pcg_s']:.0f} s for n_cg {full['n_cg']}, 1 thread, on {stored['host']['model']}) "
            f"scaled by this host's speed on a sample ({one['family']} at sides {one['sizes']}, "
            f"1 thread: {speed:.2f} x that machine's time) and to {nrhs} RHS at the GPU run's n_cg"))
        out["power_law_check"] = {"model": law_txt, "predicted_full_s": t_law_stored * speed,
                                  "measured_full_s_scaled": speed * (full["factor_s"] + full["pcg_s"]),
                                  "ratio": t_law_stored / (full["factor_s"] + full["pcg_s"])}
    else:
        out.update(value=nrhs / t_law, predicted_s_per_step=t_law, sample=(
            f"oracle on {one['family']} at sides {one['sizes']} (n={ns}), 1 thread; {law_txt} "
            f"evaluated at n={n_full} with the GPU run's n_cg x {nrhs} RHS"))
    allc = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                      os.cpu_count() or 1))
    if allc > 1:
        many = oracle_sample(workload, w, scheme, eps, allc, sizes=one["sizes"][:1])
        su = (tf[0] + ti[0]) / (many["factor_s"][0] + many["pcg_iter_s"][0])
        out["all_cores"] = {"cores": allc, "speedup_over_1": su, "value": out["value"] * su,
                            "sample_s": {k: many[k] for k in ("sizes", "factor_s", "pcg_iter_s")}}
    return out


# HBM traffic per launch of a kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) over `bench.py --steps 1 --warmup 0`,
# each scaled by what the same counter reads for a plain 256 MiB device copy.
# The figures hold only for the workload and the sources they were taken on:
# on another workload, or if any listed file has changed since, the traffic is
# reported as null.
MEASURED_TRAFFIC = {
    # (kernel, workload): HBM counters per launch (KiB, raw, averaged over the
    # kernel's launches of one factorization) from two rocprofv3 --pmc runs of
    # this script, the copy-probe scales, and the sources they were taken on
    # (profiles/ holds the commands and the full tables)
    ("k_cpqr_coop", "fv3d_128"): {
        "sources": {
            "paper_2007_00789_amd/csrc/kernels_qr_coop.hip": "1626c2057b1427c5c83788d9e9ce5e1c611f16cbe039f461e1bb73ec8c13e94f",
            "paper_2007_00789_amd/csrc/factor.cpp": "ea2695ebe9dcaf5a55635a9c43c029f245a005e6fbfd85229774c41c5cf2245c",
        },
        "fetch_kib": 78894.6, "write_kib": 447917.1,
        "fetch_scale": 1.99981, "write_scale": 1.0,
    },
    ("k_cpqr_coop", "lap3d_64"): {
        "sources": {
            "paper_2007_00789_amd/csrc/kernels_qr_coop.hip": "1626c2057b1427c5c83788d9e9ce5e1c611f16cbe039f461e1bb73ec8c13e94f",
            "paper_2007_00789_amd/csrc/factor.cpp": "ea2695ebe9dcaf5a55635a9c43c029f245a005e6fbfd85229774c41c5cf2245c",
        },
        "fetch_kib": 11358.6, "write_kib": 58176.9,
        "fetch_scale": 1.99981, "write_scale": 1.0,
    },
}


def measured_traffic(kernel, workload):
    """Calibrated HBM bytes per launch of `kernel` on `workload`, or None if not
    measured there on the current sources."""
    import hashlib
    m = MEASURED_TRAFFIC.get((kernel, workload))
    if m is None:
        return None
    for rel, digest in m["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


def bench_batch(args):
    """Batch workload: 256 independent problems (128 2D Laplacians, side
    U{32..256}; 128 anisotropic 3D operators, side U{16..48}, axis weights
    (1, 1e-2, 1e2)), each with its own depth round(log2(n/64)), eps 1e-2, SO,
    one N(0,1) right-hand side (seed 3000 + j), PCG to 1e-10.  One step =
    spand_factor + spand_pcg of the whole batch in the same launches."""
    import torch
    from paper_2007_00789_amd import spand
    from synthetic import batch_problems, rhs

    probs = batch_problems()
    tol = 1e-10
    opts = spand.make_opts(depth=0, skip=4, eps=args.eps, scheme=args.scheme)
    ctx = spand.Context(0)
    t0 = time.perf_counter()
    plan = spand.analyze_batch([(p.n, p.rowptr, p.colind, p.coords) for p in probs], opts, ctx)
    analyze_s = time.perf_counter() - t0
    vals = torch.from_numpy(np.concatenate([p.vals for p in probs])).to("cuda:0")
    b = torch.from_numpy(np.concatenate([rhs(p.n, 1, 3000 + j)[:, 0] for j, p in enumerate(probs)])).to("cuda:0")
    x = torch.zeros_like(b)

    def step():
        t = time.perf_counter()
        fac = ctx.factor(plan, vals, opts)
        tf = time.perf_counter() - t
        it, rr = ctx.pcg(fac, 1, b, x, tol, 1000)
        ts = time.perf_counter() - t - tf
        info = fac.info()
        fac.close()
        return tf, ts, it, rr, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    facs, sols = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tf, ts, it, rr, info = step()
        facs.append(tf)
        sols.append(ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    assert np.all(rr < 10 * tol), rr.max()
    nnz = sum(p.nnz for p in probs)
    out = {
        "metric": "PCG solves/s to 1e-10 rel. residual (batch of independent problems)",
        "value": len(probs) * args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(probs)} problems: 128 2D 5-point Laplacians side "
                               f"U{{32..256}}, 128 3D anisotropic (1, 1e-2, 1e2) side U{{16..48}}; "
                               f"n={plan.n}, eps {args.eps:g}, {args.scheme}, FP64, 1 RHS each, "
                               f"PCG tol {tol:g}",
                   "global_batch": len(probs), "parallelism": "single GPU"},
        "factor_ms": 1e3 * float(np.mean(facs)),
        "solve_ms": 1e3 * float(np.mean(sols)),
        "n_cg_max": int(it.max()), "n_cg_mean": float(it.mean()),
        "relres_max": float(rr.max()),
        "mu": info["nnz_L"] / nnz,
        "factor_gflop": info["flops"] / 1e9,
        "analyze_s": analyze_s,
    }
    print(json.dumps(out), flush=True)


def bench_c1grid(args):
    """The 3D 7-point Laplacian 64^3 (depth 12, skip 4, 4 RHS ~ N(0,1), seed
    2001, PCG to 1e-10) over eps in {1e-1, 1e-2, 1e-3} x {first, second order}:
    per configuration solves/s (factorization included), factor and solve time,
    n_cg, nnz(L)/nnz(A) and the true residual.  One JSON line; `value` is the
    second-order eps = 1e-2 configuration's solves/s."""
    import torch
    from paper_2007_00789_amd import spand
    from synthetic import workload, rhs

    prob, w = workload("lap3d_64")
    nrhs, tol = w["nrhs"], w["tol"]
    ctx = spand.Context(0)
    vals = torch.from_numpy(prob.vals).to("cuda:0")
    b = torch.from_numpy(np.asfortranarray(rhs(prob.n, nrhs, w["rhs_seed"])).reshape(-1, order="F").copy()).to("cuda:0")
    x = torch.zeros_like(b)
    plan = None
    rows = []
    for prec, eps, scheme in [(pr, e, sc) for pr in ("FP64", "FP32_BF16") for e in (1e-1, 1e-2, 1e-3)
                              for sc in ("FO", "SO")]:
        if True:
            opts = spand.make_opts(depth=w["depth"], skip=w["skip"], eps=eps, scheme=scheme,
                                   precision=prec)
            if plan is None:
                plan = spand.analyze(prob.n, prob.rowptr, prob.colind, prob.coords, opts, ctx)
            tfs, tss = [], []
            for i in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                fac = ctx.factor(plan, vals, opts)
                tf = time.perf_counter() - t
                it, rr = ctx.pcg(fac, nrhs, b, x, tol, 1000)
                ts = time.perf_counter() - t - tf
                info = fac.info()
                fac.close()
                if i >= args.warmup:
                    tfs.append(tf)
                    tss.append(ts)
            step = float(np.mean(tfs) + np.mean(tss))
            rows.append({"precision": prec, "eps": eps, "scheme": scheme, "solves_per_s": nrhs / step,
                         "factor_ms": 1e3 * float(np.mean(tfs)), "solve_ms": 1e3 * float(np.mean(tss)),
                         "n_cg": [int(v) for v in it], "relres_max": float(rr.max()),
                         "mu": info["nnz_L"] / prob.nnz,
                         "factor_tflops": info["flops"] / float(np.mean(tfs)) / 1e12})
    ref = [r for r in rows if r["eps"] == 1e-2 and r["scheme"] == "SO" and r["precision"] == "FP64"][0]
    for r in rows:   # the FP32 form against the FP64 one on the same (eps, scheme)
        if r["precision"] != "FP64":
            base = [q for q in rows if q["precision"] == "FP64" and q["eps"] == r["eps"]
                    and q["scheme"] == r["scheme"]][0]
            r["speedup_vs_fp64"] = r["solves_per_s"] / base["solves_per_s"]
    out = {
        "metric": "PCG solves/s to 1e-10 rel. residual; factor TFLOP/s; p50/p99 solve latency",
        "value": ref["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * nrhs / ref["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"lap3d 64^3 7-point Laplacian, n={prob.n}, depth {w['depth']}, "
                               f"skip {w['skip']}, eps x scheme x precision grid (value: FP64 SO "
                               f"eps 1e-2), {nrhs} RHS N(0,1), FP64 PCG tol {tol:g}",
                   "global_batch": nrhs, "parallelism": "single GPU"},
        "grid": rows,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Serving workload: a stream of solve requests with Poisson arrivals at
    --serve-rate per second (default 50, far above what one GPU serves, so
    the server runs saturated and requests_per_s is its saturation rate; a
    rate below it gives the latency of an unsaturated server); 3D FV diffusion matrices with side U{32..96} and k = 10^u,
    u ~ U[-2,2] per cell; 1..16 N(0,1) right-hand sides per request; about 30%
    of the requests reuse the matrix of an earlier one (synthetic.serve_stream).
    Requests are submitted at their arrival times to the library's server
    (spand_server_*: continuous batching of new matrices into one analysis and
    factorization per slot, resident factors, one PCG per factor and slot).
    One step = one request; value = right-hand sides solved to 1e-10 per second
    over the stream's makespan (first arrival to last completion)."""
    import torch
    from paper_2007_00789_amd import spand
    from synthetic import serve_stream, fv_diffusion_3d, laplacian_3d, rhs

    tol = 1e-10
    stream = serve_stream(count=args.serve_count, rate=args.serve_rate)
    mats = {}
    for r in stream:
        if r["key"] not in mats:
            mats[r["key"]] = fv_diffusion_3d(r["side"], r["umax"], r["mseed"])
    bs = [rhs(mats[r["key"]].n, r["nrhs"], r["rhs_seed"]) for r in stream]
    opts = spand.make_opts(depth=0, skip=4, eps=args.eps, scheme=args.scheme)
    # warm-up: load the device code once, outside the stream
    w = laplacian_3d(16)
    with spand.Server(opts, tol=tol, slots=1) as srv:
        srv.result(srv.submit(-1, rhs(w.n, 1, 1), (w.n, w.rowptr, w.colind, w.coords, w.vals)))
    torch.cuda.synchronize()
    seen = set()
    handles, t_sub = [], []
    with spand.Server(opts, tol=tol, maxit=1000, max_bytes=args.serve_bytes << 30,
                      slots=args.serve_slots, max_batch=args.serve_batch) as srv:
        t0 = time.perf_counter()
        for r, b in zip(stream, bs):
            delay = t0 + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            key = r["side"] * 1_000_000 + r["mseed"]
            m = mats[r["key"]]
            mat = None if key in seen else (m.n, m.rowptr, m.colind, m.coords, m.vals)
            seen.add(key)
            t_sub.append(time.perf_counter())
            handles.append(srv.submit(key, b, mat))
        res = [srv.result(h, check=False) for h in handles]
        stats = srv.stats()
    lat = np.array([q[3] for q in res])
    done = np.array(t_sub) + lat
    makespan = float(done.max() - t0)
    cols = sum(r["nrhs"] for r in stream)
    iters = np.concatenate([q[1] for q in res])
    rel = np.concatenate([q[2] for q in res])
    assert all(q[4] == spand.SPAND_OK for q in res), [q[4] for q in res]
    assert np.all(rel < 10 * tol), rel.max()
    n_reuse = len(stream) - len(mats)
    out = {
        "metric": "PCG solves/s to 1e-10 rel. residual; p50/p99 request latency (serving stream)",
        "value": cols / makespan,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(stream),
        "warmup": 1,
        "ms_per_step": 1e3 * makespan / len(stream),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving stream of {len(stream)} requests, Poisson arrivals at "
                               f"{args.serve_rate:g}/s; "
                               f"3D FV diffusion side U{{32..96}}, k = 10^U[-2,2]; 1-16 RHS N(0,1); "
                               f"{n_reuse} requests reuse a factor; eps {args.eps:g}, {args.scheme}, "
                               f"FP64, PCG tol {tol:g}; {args.serve_slots} slots, "
                               f"batch <= {args.serve_batch}, budget {args.serve_bytes} GiB",
                   "global_batch": len(stream), "parallelism": "single GPU"},
        "requests_per_s": len(stream) / makespan,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "arrival_span_s": float(stream[-1]["t"]),
        "makespan_s": makespan,
        "rhs_total": cols,
        "n_cg_max": int(iters.max()), "n_cg_mean": float(iters.mean()),
        "relres_max": float(rel.max()),
        "server": stats,
    }
    print(json.dumps(out), flush=True)


def bench_eig2d(args):
    """Forward-error study on the 2D constant-coefficient Poisson problem
    (Sec. 4): d = 1000 grid (n = 10^6, depth 14, skip 4), modes
    p = floor(1.25^k) <= d, errors ||(I - M A) v_p||_2 for FO and SO at
    eps = 0.1 and 0.01.  A v_p is formed on the host (closed-form input); each
    factorization applies M to all modes at once on the device."""
    import torch
    from paper_2007_00789_amd import spand
    from synthetic import laplacian_2d, poisson_modes, poisson_eigvec

    d = args.eig_d
    depth = max(0, int(round(np.log2(d * d / 64.0))))
    prob = laplacian_2d(d)
    ps = poisson_modes(d)
    V = np.stack([poisson_eigvec(d, q)[0] for q in ps], 1)
    lam = [poisson_eigvec(d, q)[1] for q in ps]
    AV = prob.scipy() @ V
    nm = len(ps)
    ctx = spand.Context(0)
    dx = torch.from_numpy(np.asfortranarray(AV).reshape(-1, order="F").copy()).to("cuda:0")
    dy = torch.zeros_like(dx)
    vals = torch.from_numpy(prob.vals).to("cuda:0")
    errs, times = {}, {}
    plan = None
    for eps in (0.1, 0.01):
        for scheme in ("FO", "SO"):
            opts = spand.make_opts(depth=depth, skip=4, eps=eps, scheme=scheme)
            if plan is None:
                plan = spand.analyze(prob.n, prob.rowptr, prob.colind, prob.coords, opts, ctx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac = ctx.factor(plan, vals, opts)
            t1 = time.perf_counter()
            ctx.apply(fac, nm, dx, dy)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            Z = dy.cpu().numpy().reshape(prob.n, nm, order="F")
            errs[f"{scheme}_{eps:g}"] = np.linalg.norm(V - Z, axis=0).tolist()
            times[f"{scheme}_{eps:g}"] = {"factor_ms": 1e3 * (t1 - t0), "apply_ms": 1e3 * (t2 - t1),
                                          "mu": fac.info()["nnz_L"] / prob.nnz}
            fac.close()
    better = [so < fo for e in ("0.1", "0.01")
              for so, fo in zip(errs[f"SO_{e}"], errs[f"FO_{e}"])]
    mid = [i for i, l in enumerate(lam) if l >= 1e-2]
    ratio = float(np.exp(np.mean([np.log(errs["SO_0.1"][i] / errs["FO_0.01"][i]) for i in mid])))
    out = {
        "metric": "forward error ||(I - M A) v||_2 on unit eigenvectors, 2D Poisson",
        "value": float(np.mean(better)),
        "unit": "fraction of (mode, eps) with SO error below FO error",
        "n_gpus": 1, "steps": 4, "warmup": 0, "higher_is_better": True, "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D 5-point Poisson {d}x{d}, n={prob.n}, depth {depth}, skip 4, "
                               f"modes p = floor(1.25^k) <= {d} ({nm} modes)"},
        "modes": ps, "eigenvalues": lam, "errors": errs, "timing": times,
        "so_eps0.1_over_fo_eps0.01_geomean_lambda_ge_1e-2": ratio,
    }
    print(json.dumps(out), flush=True)


def bench_table1(args):
    """Scaling study on 2D Laplacians (the paper's Table 1 setting): d x d
    grids, d = 400 ... d_max doubling, contrast rho in {1, 100} (the field of
    synthetic.high_contrast_2d, seed 5000 + d; rho = 1 is the constant
    coefficient case), b = ones, eps in {0.01, 0.001}, FO and SO, depth
    round(log2(n/64)), skip 4, PCG to 1e-10.  Reports mu, n_cg, factor and
    solve seconds per run (device times; the analysis per grid is separate)."""
    import torch
    from paper_2007_00789_amd import spand
    from synthetic import high_contrast_2d

    rows = []
    ctx = spand.Context(0)
    d = 400
    while d <= args.table1_dmax:
        for rho in (1.0, 100.0):
            prob = high_contrast_2d(d, rho, seed=5000 + d)
            depth = max(0, int(round(np.log2(prob.n / 64.0))))
            t0 = time.perf_counter()
            plan = spand.analyze(prob.n, prob.rowptr, prob.colind, prob.coords,
                                 spand.make_opts(depth=depth, skip=4), ctx)
            analyze_s = time.perf_counter() - t0
            vals = torch.from_numpy(prob.vals).to("cuda:0")
            b = torch.ones(prob.n, dtype=torch.float64, device="cuda:0")
            x = torch.zeros_like(b)
            for eps in (0.01, 0.001):
                for scheme in ("FO", "SO"):
                    opts = spand.make_opts(depth=depth, skip=4, eps=eps, scheme=scheme)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    fac = ctx.factor(plan, vals, opts)
                    t2 = time.perf_counter()
                    it, rr = ctx.pcg(fac, 1, b, x, 1e-10, 1000)
                    t3 = time.perf_counter()
                    # PCG stops on the recursive residual (the paper's rule);
                    # relres is the true residual at exit, which can stay
                    # above the tolerance when kappa(A) is large
                    row = {"d": d, "n": prob.n, "rho": rho, "eps": eps, "scheme": scheme,
                           "mu": fac.info()["nnz_L"] / prob.nnz, "n_cg": int(it[0]),
                           "relres": float(rr[0]), "true_residual_below_tol": bool(rr[0] < 1e-10),
                           "T_f": t2 - t1, "T_s": t3 - t2, "analyze_s": analyze_s}
                    rows.append(row)
                    print(json.dumps(row), file=sys.stderr, flush=True)
                    fac.close()
            plan.close()
            del vals, b, x
        d *= 2
    ratios = {}
    for r in rows:
        if r["scheme"] == "SO":
            fo = next(q for q in rows if q["scheme"] == "FO" and
                      (q["d"], q["rho"], q["eps"]) == (r["d"], r["rho"], r["eps"]))
            ratios[f"d{r['d']}_rho{r['rho']:g}_eps{r['eps']:g}"] = r["n_cg"] / fo["n_cg"]
    out = {
        "metric": "PCG iterations SO / FO on 2D Laplacians (scaling study)",
        "value": float(np.mean(list(ratios.values()))),
        "unit": "mean n_cg ratio SO/FO",
        "n_gpus": 1, "steps": len(rows), "warmup": 0, "higher_is_better": False,
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D 5-point, d = 400..{args.table1_dmax}, rho in {{1, 100}}, "
                               "b = ones, eps in {0.01, 0.001}, skip 4, PCG tol 1e-10"},
        "ratios": ratios, "rows": rows,
        "rows_true_residual_above_tol": [
            f"d{r['d']}_rho{r['rho']:g}_eps{r['eps']:g}_{r['scheme']}: {r['relres']:.2e}"
            for r in rows if not r["true_residual_below_tol"]],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--scheme", default="SO")
    ap.add_argument("--precision", default="FP64", choices=["FP64", "FP32", "FP32_BF16"],
                    help="arithmetic of the factorization (PCG is FP64 in every mode)")
    ap.add_argument("--apply-graph", type=int, default=0,
                    help="1: the apply captured in a HIP graph and replayed by PCG")
    ap.add_argument("--prescale", type=int, default=0,
                    help="1: factor D^-1/2 A D^-1/2 (symmetric diagonal prescaling)")
    ap.add_argument("--workload", default="fv3d_128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-count", type=int, default=48, help="requests of the serving stream")
    ap.add_argument("--eig-d", type=int, default=1000, help="grid side of the eigenvector study")
    ap.add_argument("--table1-dmax", type=int, default=3200, help="largest grid side of the scaling study")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-rate", type=float, default=50.0, help="request arrivals per second")
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--serve-bytes", type=int, default=200, help="factor budget, GiB")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the factorization and PCG run on a single MI355X "
              "(independent problems would shard whole, one problem along its nested-"
              "dissection tree); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        return bench_batch(args)
    if args.workload == "c1grid":
        return bench_c1grid(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "eig2d":
        return bench_eig2d(args)
    if args.workload == "table1":
        return bench_table1(args)

    import torch
    from paper_2007_00789_amd import spand
    from synthetic import workload, rhs

    prob, w = workload(args.workload)
    nrhs, tol = w["nrhs"], w["tol"]
    opts = spand.make_opts(depth=w["depth"], skip=w["skip"], eps=args.eps, scheme=args.scheme,
                           precision=args.precision, prescale=args.prescale,
                           apply_graph=args.apply_graph)
    ctx = spand.Context(0)
    t0 = time.perf_counter()
    plan = spand.analyze(prob.n, prob.rowptr, prob.colind, prob.coords, opts, ctx)
    analyze_s = time.perf_counter() - t0
    vals = torch.from_numpy(prob.vals).to("cuda:0")
    b = torch.from_numpy(np.asfortranarray(rhs(prob.n, nrhs, w["rhs_seed"])).reshape(-1, order="F").copy()).to("cuda:0")
    x = torch.zeros_like(b)

    def step():
        t = time.perf_counter()
        fac = ctx.factor(plan, vals, opts)
        tf = time.perf_counter() - t
        it, rr = ctx.pcg(fac, nrhs, b, x, tol, 1000)
        ts = time.perf_counter() - t - tf
        info = fac.info()
        fac.close()
        return tf, ts, it, rr, info

    # warm-up; the last warm-up step records every kernel's event time (the
    # per-kernel breakdown), the timed steps only the dominant kernel's
    for wi in range(args.warmup):
        if wi == args.warmup - 1:
            torch.cuda.synchronize()
            ctx.profile(True)
        step()
    torch.cuda.synchronize()
    breakdown = ctx.profile_entries() if args.warmup > 0 else {}
    ctx.profile(False)
    dom = max(breakdown.items(), key=lambda kv: kv[1][0])[0] if breakdown else None
    ctx.profile(True, only=dom)
    times, facs, sols, iters, relres = [], [], [], [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tf, ts, it, rr, info = step()
        facs.append(tf)
        sols.append(ts)
        iters.append(it.copy())
        relres.append(rr.copy())
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    prof = ctx.profile_entries()
    ctx.profile(False)

    ms_per_step = 1e3 * total / args.steps
    value = nrhs * args.steps / total
    flops = info["flops"]
    factor_tflops = flops / np.mean(facs) / 1e12
    it_all = np.concatenate(iters)
    assert np.all(np.concatenate(relres) < 10 * tol), relres

    # dominant kernel: the largest event time of the warm-up step (every
    # kernel timed when there is no warm-up); its launches are timed live
    # in the timed region
    per = 1
    if dom is None:
        breakdown, per = prof, args.steps
        dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    dms, dcalls, dwork = prof[dom]
    kernel_ms = {k: round(v[0] / per, 3) for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1][0])}
    if dom in ("k_cpqr", "k_cpqr_coop"):
        # FP64 vector ALU work of the pivoted QR: sum over reflectors of 4(a-j)(k-j)
        ach = dwork / (dms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                "work": "FP64 flops of the pivoted QR, sum over reflectors j of 4(a-j)(k-j)",
                "limiter": "latency of the dependent pivot steps (one reduction, barrier and "
                           "rank-1 update per reflector), not the ALU rate",
                "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "traffic": measured_traffic(dom, args.workload),
                "avg_launch_ms": dms / dcalls, "launches": dcalls}
    else:
        roof = {"bound": None, "kernel": dom, "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None, "avg_launch_ms": dms / dcalls, "launches": dcalls}

    out = {
        "metric": "PCG solves/s to 1e-10 rel. residual; factor TFLOP/s; p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD_NAMES.get(args.workload, args.workload)}, n={prob.n}, "
                               f"depth {w['depth']}, skip {w['skip']}, eps {args.eps:g}, "
                               f"{args.scheme}, {args.precision} factor"
                               f"{', D^-1/2 prescaling' if args.prescale else ''}, FP64 PCG, {nrhs} RHS "
                               f"N(0,1), PCG tol {tol:g}",
                   "global_batch": nrhs, "parallelism": "single GPU"},
        "factor_tflops": factor_tflops,
        "factor_ms": 1e3 * float(np.mean(facs)),
        "solve_ms": 1e3 * float(np.mean(sols)),
        "latency_ms_p50": 1e3 * float(np.percentile(np.add(facs, sols), 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(np.add(facs, sols), 99)),
        "n_cg": [int(v) for v in iters[-1]],
        "relres_max": float(np.max(np.concatenate(relres))),
        "mu": info["nnz_L"] / prob.nnz,
        "factor_gflop": flops / 1e9,
        "analyze_s": analyze_s,
        "kernel_ms_per_step": kernel_ms,
        "kernel_work": kernel_work(breakdown, per, args.precision),
        "gemm_tiles": ctx.gemm_tuning(0 if args.precision == "FP64" else 1),
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.workload in CPU_SAMPLE:
        out["cpu_baseline"] = cpu_baseline(args.workload, w, prob.n, args.scheme, args.eps,
                                           iters[-1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
