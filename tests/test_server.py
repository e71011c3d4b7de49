"""Serving loop: requests on new and resident factors, continuous batching.

Host checks (no GPU): argument validation of spand_server_create.

GPU checks: a mixed stream of requests (several matrices, repeated keys,
1-3 right-hand sides, submitted in bursts while earlier ones run) gives for
every request the result the same request gets alone -- spand_analyze +
spand_factor + spand_pcg on its matrix only -- and the oracle's: iteration
counts within 1, solutions within 1e-10 relative.  A byte budget below the
footprint of two factors forces factors out and back in, with the same
results.
"""
import ctypes as C

import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d, rhs
from oracle import nd, spand as ospand, pcg as opcg

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

SKIP = 1
EPS = 1e-2
TOL = 1e-10

MATRICES = {
    11: lambda: laplacian_2d(40),
    12: lambda: laplacian_3d(12),
    13: lambda: fv_diffusion_3d(10, 2.0, 7),
    14: lambda: laplacian_2d(27, 19),
    15: lambda: fv_diffusion_3d(12, 2.0, 8),
}
# (key, nrhs, rhs seed); bursts are submitted together, each after the
# previous burst's first request has finished
BURSTS = [
    [(11, 1, 500), (12, 2, 501), (13, 1, 502)],
    [(11, 3, 503), (14, 1, 504), (12, 1, 505), (15, 2, 506)],
    [(13, 2, 507), (15, 1, 508), (11, 1, 509), (14, 2, 510), (12, 3, 511)],
]


def _lib():
    from paper_2007_00789_amd import spand
    try:
        spand.load()
    except OSError:
        pytest.skip("libspand.so not built")
    return spand


def test_server_create_rejects_bad_arguments():
    spand = _lib()
    lib = spand.load()
    opts = spand.make_opts(skip=SKIP, eps=EPS)
    h = C.c_void_p()
    for args in [(0, 1e-10, 100, 1 << 30, 0, 4), (0, 1e-10, 100, 1 << 30, 17, 4),
                 (0, 0.0, 100, 1 << 30, 1, 4), (0, 1e-10, 0, 1 << 30, 1, 4),
                 (0, 1e-10, 100, 0, 1, 4), (0, 1e-10, 100, 1 << 30, 1, 0),
                 (-1, 1e-10, 100, 1 << 30, 1, 4)]:
        dev, tol, maxit, mb, slots, mbatch = args
        st = lib.spand_server_create(dev, C.byref(opts), tol, maxit, mb, slots, mbatch,
                                     C.byref(h))
        assert st != spand.SPAND_OK, args
        assert not h.value
    if not torch.cuda.is_available():
        st = lib.spand_server_create(0, C.byref(opts), 1e-10, 100, 1 << 30, 1, 4, C.byref(h))
        assert st != spand.SPAND_OK and not h.value


def _solo(spand, ctx, p, nrhs, seed):
    """The request alone: its own plan, factor and PCG."""
    opts = spand.make_opts(skip=SKIP, eps=EPS)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts)
    fac = ctx.factor(plan, torch.from_numpy(p.vals).cuda(), opts)
    b = rhs(p.n, nrhs, seed)
    db = torch.from_numpy(b.reshape(-1, order="F").copy()).cuda()
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, nrhs, db, dx, TOL, 1000)
    x = dx.cpu().numpy().reshape(p.n, nrhs, order="F")
    depth = plan.depth
    fac.close()
    plan.close()
    return x, it, depth


def _run_stream(spand, server, probs):
    results = {}
    seen = set()
    for burst in BURSTS:
        reqs = []
        for key, nrhs, seed in burst:
            p = probs[key]
            mat = None if key in seen else (p.n, p.rowptr, p.colind, p.coords, p.vals)
            seen.add(key)
            reqs.append(((key, nrhs, seed), server.submit(key, rhs(p.n, nrhs, seed), mat)))
        # the next burst arrives while the rest of this one is still running
        first, req = reqs[0]
        results[first] = server.result(req)
        for tag, req in reqs[1:]:
            results[tag] = server.result(req)
    return results


def _check(spand, results, probs):
    ctx = spand.Context(0)
    oracle = {}
    for (key, nrhs, seed), (x, it, rr, lat, st) in results.items():
        p = probs[key]
        print("request", key, nrhs, seed, flush=True)
        assert st == spand.SPAND_OK
        assert lat > 0
        xs, its, depth = _solo(spand, ctx, p, nrhs, seed)
        if key not in oracle:
            plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, SKIP)
            oracle[key] = ospand.factor(p.scipy(), plan_o, EPS, "SO")
        A = p.scipy()
        F = oracle[key]
        Xo, itso, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v),
                                     rhs(p.n, nrhs, seed), TOL)
        for j in range(nrhs):
            assert rr[j] < TOL
            assert abs(int(it[j]) - int(its[j])) <= 1, (key, j)
            assert abs(int(it[j]) - int(itso[j])) <= 1, (key, j)
            assert np.linalg.norm(x[:, j] - xs[:, j]) <= 1e-10 * np.linalg.norm(xs[:, j])
            assert np.linalg.norm(x[:, j] - Xo[:, j]) <= 1e-10 * np.linalg.norm(Xo[:, j])
    ctx.close()


@gpu
def test_server_results_match_solo_solves():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spand = _lib()
    probs = {k: make() for k, make in MATRICES.items()}
    opts = spand.make_opts(skip=SKIP, eps=EPS)
    with spand.Server(opts, tol=TOL, maxit=1000, slots=2, max_batch=4) as srv:
        results = _run_stream(spand, srv, probs)
        stats = srv.stats()
    print(stats, flush=True)
    # every matrix factored once (the budget holds them all), fewer PCG calls
    # than requests when requests were batched
    assert stats["factored_matrices"] == len(MATRICES)
    assert stats["queued"] == 0
    _check(spand, results, probs)


@gpu
def test_server_budget_releases_and_refactors():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spand = _lib()
    probs = {k: make() for k, make in MATRICES.items()}
    opts = spand.make_opts(skip=SKIP, eps=EPS)
    # a budget that holds about one of these factors at a time
    budget = max(len(p.colind) for p in probs.values()) * 96 * 8 + 1
    with spand.Server(opts, tol=TOL, maxit=1000, slots=2, max_batch=4,
                      max_bytes=budget) as srv:
        results = _run_stream(spand, srv, probs)
        stats = srv.stats()
    print(stats, flush=True)
    assert stats["factored_matrices"] > len(MATRICES)
    _check(spand, results, probs)
