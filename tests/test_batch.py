"""Multi-problem batching: one plan for several independent problems.

Host checks (no GPU): the batch plan is the block-diagonal union of the
problems' own plans with their levels aligned at the leaves (problem i's step l
is batch step l + D - D_i, interiors of all problems before interfaces, each
problem's clusters in its own canonical order).

GPU checks: every problem's ranks in the batch factorization equal the
oracle's for that problem alone (bit-exact), and the batched PCG (one CG per
problem and column) matches the oracle's iteration counts and solutions.
"""
import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d, rhs
from oracle import nd, spand as ospand, pcg as opcg

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

# (problem, depth): different sizes, dimensions and depths
PROBLEMS = [
    (lambda: laplacian_2d(40), 5),
    (lambda: laplacian_3d(12), 4),
    (lambda: fv_diffusion_3d(10, 2.0, 7), 3),
    (lambda: laplacian_2d(27, 19), 6),
]
SKIP = 1
EPS = 1e-2


def _lib():
    from paper_2007_00789_amd import spand
    try:
        spand.load()
    except OSError:
        pytest.skip("libspand.so not built")
    return spand


def _plans(spand):
    probs = [make() for make, _ in PROBLEMS]
    depths = [d for _, d in PROBLEMS]
    opts = spand.make_opts(skip=SKIP, eps=EPS, scheme="SO")
    batch = spand.analyze_batch([(p.n, p.rowptr, p.colind, p.coords) for p in probs], opts,
                                depths=depths)
    solo = []
    for p, d in zip(probs, depths):
        o = spand.make_opts(depth=d, skip=SKIP, eps=EPS, scheme="SO")
        solo.append(spand.analyze(p.n, p.rowptr, p.colind, p.coords, o))
    return probs, depths, batch, solo


def _maps(batch, solo, depths):
    """For every batch step: per problem (own step, interior offset, interface offset)."""
    D = max(depths)
    out = {}
    for lm in range(D + 1):
        st = batch.step(lm)
        rows, io, fo = [], 0, 0
        for pl, d in zip(solo, depths):
            l = lm - (D - d)
            if l < 0:
                rows.append(None)
                continue
            s = pl.step(l)
            rows.append((l, io, fo, s))
            io += s["n_interior"]
            fo += s["n_clusters"] - s["n_interior"]
        assert io == st["n_interior"] and io + fo == st["n_clusters"], lm
        out[lm] = (st, rows)
    return out


def test_batch_plan_is_the_union_of_the_problems_plans():
    spand = _lib()
    probs, depths, batch, solo = _plans(spand)
    cnt, off = batch.segments()
    assert cnt == len(probs)
    assert list(np.diff(off)) == [p.n for p in probs]
    D = max(depths)
    assert batch.depth == D
    for lm, (st, rows) in _maps(batch, solo, depths).items():
        assert st["sparsified"] == (1 <= lm <= D - SKIP)
        nI = st["n_interior"]
        for i, row in enumerate(rows):
            if row is None:
                continue
            l, io, fo, s = row
            own_nI = s["n_interior"]

            def m(c):
                return io + c if c < own_nI else nI + fo + (c - own_nI)

            for c in range(s["n_clusters"]):
                x = m(c)
                got = st["adj"][st["adj_ptr"][x]:st["adj_ptr"][x + 1]]
                exp = [m(q) for q in s["adj"][s["adj_ptr"][c]:s["adj_ptr"][c + 1]]]
                assert list(got) == exp, (lm, i, c)
                assert st["colour"][x] == s["colour"][c]
                if lm < D:
                    gch = st["child"][st["child_ptr"][x]:st["child_ptr"][x + 1]]
                    nxt = _maps(batch, solo, depths)[lm + 1][1][i]
                    _, io2, fo2, s2 = nxt
                    nI2 = batch.step(lm + 1)["n_interior"]
                    ech = [io2 + q if q < s2["n_interior"] else nI2 + fo2 + (q - s2["n_interior"])
                           for q in s["child"][s["child_ptr"][c]:s["child_ptr"][c + 1]]]
                    assert list(gch) == ech, (lm, i, c)


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a).reshape(-1, order="F").copy()).to("cuda")


@gpu
def test_batched_factor_and_pcg_match_the_oracle_per_problem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spand = _lib()
    probs, depths, batch, solo = _plans(spand)
    ctx = spand.Context(0)
    print("batch of", len(probs), "problems", flush=True)
    opts = spand.make_opts(skip=SKIP, eps=EPS, scheme="SO")
    vals = np.concatenate([p.vals for p in probs])
    fac = ctx.factor(batch, _dev(vals), opts)
    maps = _maps(batch, solo, depths)
    nrhs, tol = 2, 1e-10
    bs, xs_ref, its_ref = [], [], []
    for i, (p, d) in enumerate(zip(probs, depths)):
        plan_o = nd.analyze(p.rowptr, p.colind, p.coords, d, SKIP)
        F = ospand.factor(p.scipy(), plan_o, EPS, "SO")
        D = max(depths)
        for l, recs in F.ranks.items():
            lm = l + D - d
            st, rows = maps[lm]
            _, io, fo, s = rows[i]
            got = fac.ranks(lm, st["n_clusters"])
            for (c, a, k, r, r2) in recs:
                x = io + c if c < s["n_interior"] else st["n_interior"] + fo + (c - s["n_interior"])
                assert (got["a"][x], got["k"][x], got["r"][x], got["r2"][x]) == (a, k, r, r2), (i, l, c)
        b = rhs(p.n, nrhs, 100 + i)
        A = p.scipy()
        X, its, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
        bs.append(b)
        xs_ref.append(X)
        its_ref.append(its)
    b_all = np.concatenate(bs, axis=0)
    db = _dev(b_all)
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, nrhs, db, dx, tol, 1000)
    x_all = dx.cpu().numpy().reshape(b_all.shape[0], nrhs, order="F")
    _, off = batch.segments()
    for i in range(len(probs)):
        xi = x_all[off[i]:off[i + 1]]
        for j in range(nrhs):
            assert abs(int(it[i, j]) - its_ref[i][j]) <= 1, (i, j)
            assert rr[i, j] < tol
            assert np.linalg.norm(xi[:, j] - xs_ref[i][:, j]) <= 1e-10 * np.linalg.norm(xs_ref[i][:, j])


@gpu
def test_factor_batch_handles_match_the_oracle_per_problem():
    """spand_factor_batch over separately analysed plans: every handle reports
    its own problem's ranks (bit-exact against the oracle for that problem
    alone); spand_pcg_batch with different column counts per problem matches
    the oracle's iterations (+-1) and solutions (1e-10); spand_pcg and
    spand_apply on one handle give that problem's results alone."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spand = _lib()
    probs = [make() for make, _ in PROBLEMS]
    depths = [d for _, d in PROBLEMS]
    ctx = spand.Context(0)
    print("factor_batch of", len(probs), "problems", flush=True)
    plans = [spand.analyze(p.n, p.rowptr, p.colind, p.coords,
                           spand.make_opts(depth=d, skip=SKIP, eps=EPS, scheme="SO"))
             for p, d in zip(probs, depths)]
    opts = spand.make_opts(skip=SKIP, eps=EPS, scheme="SO")
    facs = ctx.factor_batch(plans, [_dev(p.vals) for p in probs], opts)
    facs2 = ctx.factor_batch(plans, [_dev(p.vals) for p in probs], opts)   # cached merged plan
    nrhs = [1, 3, 2, 1]
    tol = 1e-10
    bs, xs, refs = [], [], []
    for i, (p, d) in enumerate(zip(probs, depths)):
        plan_o = nd.analyze(p.rowptr, p.colind, p.coords, d, SKIP)
        F = ospand.factor(p.scipy(), plan_o, EPS, "SO")
        for fset in (facs, facs2):
            for l, recs in F.ranks.items():
                got = fset[i].ranks(l, plan_o.steps[l].n_clusters)
                for (c, a, k, r, r2) in recs:
                    assert (got["a"][c], got["k"][c], got["r"][c], got["r2"][c]) == (a, k, r, r2), (i, l, c)
        b = rhs(p.n, nrhs[i], 200 + i)
        A = p.scipy()
        X, its, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
        refs.append((X, its, ospand.apply(F, b[:, 0])))
        bs.append(_dev(b))
        xs.append(torch.zeros(p.n * nrhs[i], dtype=torch.float64, device="cuda"))
    res = ctx.pcg_batch(facs, nrhs, bs, xs, tol, 1000)
    for i, p in enumerate(probs):
        X, its, _ = refs[i]
        x = xs[i].cpu().numpy().reshape(p.n, nrhs[i], order="F")
        it, rr = res[i]
        for j in range(nrhs[i]):
            assert abs(int(it[j]) - its[j]) <= 1, (i, j)
            assert rr[j] < tol
            assert np.linalg.norm(x[:, j] - X[:, j]) <= 1e-10 * np.linalg.norm(X[:, j]), (i, j)
    # one handle alone: PCG and apply on its own vectors
    i = 2
    p = probs[i]
    X, its, y_ref = refs[i]
    dx = torch.zeros(p.n * nrhs[i], dtype=torch.float64, device="cuda")
    it, rr = ctx.pcg(facs2[i], nrhs[i], bs[i], dx, tol, 1000)
    x = dx.cpu().numpy().reshape(p.n, nrhs[i], order="F")
    for j in range(nrhs[i]):
        assert abs(int(it[j]) - its[j]) <= 1
        assert np.linalg.norm(x[:, j] - X[:, j]) <= 1e-10 * np.linalg.norm(X[:, j])
    dy = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    ctx.apply(facs2[i], 1, bs[i][:p.n].contiguous(), dy)
    assert np.linalg.norm(dy.cpu().numpy() - y_ref) <= 1e-11 * np.linalg.norm(y_ref)
    for f in facs + facs2:
        f.close()


@gpu
def test_hbm_budget_is_enforced():
    """opts.hbm_budget_bytes: a budget below the factor's footprint fails with
    SPAND_E_OOM; the context stays usable and an unlimited factorization of
    the same plan then succeeds."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spand = _lib()
    p = laplacian_3d(16)
    ctx = spand.Context(0)
    o = spand.make_opts(depth=6, skip=2, eps=1e-2, scheme="SO", hbm_budget_bytes=1 << 16)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, o)
    with pytest.raises(spand.SpandError) as e:
        ctx.factor(plan, _dev(p.vals), o)
    assert e.value.status == -5 and "hbm_budget_bytes" in e.value.message
    o.hbm_budget_bytes = 0
    fac = ctx.factor(plan, _dev(p.vals), o)
    assert fac.info()["factor_bytes"] > (1 << 16)
    fac.close()
