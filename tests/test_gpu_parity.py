"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (FP64):
* ordering, clusters and ranks: bit-exact (ranks of every sparsified step);
* blocks after a step's sparsification: 1e-11 relative to the block norm;
* y = M x: 1e-11 relative;
* PCG: iteration count within +-1 (identical expected) and the solution within
  1e-10 relative of the oracle's;
* eps = 0 reproduces the exact nested-dissection Cholesky (one apply solves).
"""
import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d, high_contrast_2d, rhs
from oracle import nd, spand as ospand, pcg as opcg

gpu = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a).reshape(-1, order="F").copy()).to("cuda")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_00789_amd import spand
    return spand.Context(0)


def _gpu_factor(ctx, p, depth, skip, eps, scheme, stop=-1, qr_group=0, qr_list_cap=-1,
                qr_xcd_local=1, qr_lds_cols=0, qr_single_launch=1):
    from paper_2007_00789_amd import spand
    opts = spand.make_opts(depth=depth, skip=skip, eps=eps, scheme=scheme, debug_stop_step=stop,
                           qr_lds_cols=qr_lds_cols, qr_single_launch=qr_single_launch,
                           qr_group=qr_group, qr_list_cap=qr_list_cap, qr_xcd_local=qr_xcd_local)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    vals = _dev(p.vals)
    fac = ctx.factor(plan, vals, opts)
    return plan, fac


def _oracle_ranks(F):
    out = {}
    for l, recs in F.ranks.items():
        out[l] = {p: (a, k, r, r2) for (p, a, k, r, r2) in recs}
    return out


CASES = [
    ("lap2d_64", lambda: laplacian_2d(64), 6, 4, 1e-2),
    ("lap2d_64_skip0", lambda: laplacian_2d(64), 6, 0, 1e-2),
    ("lap2d_ragged", lambda: laplacian_2d(45, 29), 6, 1, 3e-2),
    ("lap3d_16", lambda: laplacian_3d(16), 6, 1, 1e-2),
    ("fv3d_12", lambda: fv_diffusion_3d(12, 3.0, 1002), 5, 0, 1e-2),
    ("lap3d_24_eps1e-3", lambda: laplacian_3d(24), 8, 2, 1e-3),
]


@gpu
@pytest.mark.parametrize("scheme", ["FO", "SO", "SF"])
@pytest.mark.parametrize("name,make,depth,skip,eps", CASES, ids=[c[0] for c in CASES])
def test_ranks_and_memory_match_oracle(ctx, name, make, depth, skip, eps, scheme):
    p = make()
    print(f"case {name} {scheme}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, scheme)
    plan, fac = _gpu_factor(ctx, p, depth, skip, eps, scheme)
    ref = _oracle_ranks(F)
    for l in range(depth, 0, -1):
        st = plan_o.steps[l]
        got = fac.ranks(l, st.n_clusters)
        if not st.sparsified:
            assert (got["r"] == -1).all()
            continue
        for p_, (a, k, r, r2) in ref[l].items():
            assert (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2), \
                (l, p_)
    info = fac.info()
    assert info["nnz_L"] == F.nnz_L
    assert info["flops"] == pytest.approx(sum(F.flops.values()), rel=1e-12)


@gpu
@pytest.mark.parametrize("stop", [6, 5, 3, 2])
def test_blocks_after_a_step(ctx, stop):
    p = laplacian_2d(64)
    depth, skip, eps = 6, 0, 1e-2
    print(f"blocks after step {stop}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    _, B, sizes = ospand.factor(p.scipy(), plan_o, eps, "SO", stop_after=stop)
    _, fac = _gpu_factor(ctx, p, depth, skip, eps, "SO", stop=stop)
    st = plan_o.steps[stop]
    nmax = 0
    for (i, j), blk in B.items():
        got = fac.debug_block(i, j)
        assert got.shape == blk.shape, (i, j)
        if blk.size:
            scale = max(np.abs(blk).max(), 1.0)
            assert np.abs(got - blk).max() <= 1e-11 * scale, (i, j)
            nmax += 1
    assert nmax > 0
    assert all(sizes[c] == fac.debug_block(c, c).shape[0] for c in range(st.n_interior, st.n_clusters))


@gpu
@pytest.mark.parametrize("scheme", ["FO", "SO", "SF"])
@pytest.mark.parametrize("name,make,depth,skip,eps", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_apply_matches_oracle(ctx, name, make, depth, skip, eps, scheme):
    p = make()
    print(f"apply {name} {scheme}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, scheme)
    _, fac = _gpu_factor(ctx, p, depth, skip, eps, scheme)
    x = rhs(p.n, 3, 11)
    y_ref = ospand.apply(F, x)
    dx = _dev(x)
    dy = torch.zeros_like(dx)
    ctx.apply(fac, 3, dx, dy)
    y = dy.cpu().numpy().reshape(p.n, 3, order="F")
    assert np.linalg.norm(y - y_ref) <= 1e-11 * np.linalg.norm(y_ref)


@gpu
def test_apply_many_columns_in_chunks(ctx):
    """More right-hand sides than the apply kernels stage in LDS at once: the
    columns are processed in chunks, each column as in a narrow apply."""
    p = laplacian_3d(16)
    nrhs = 100
    print(f"apply lap3d_16 SO nrhs {nrhs}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, 6, 1)
    F = ospand.factor(p.scipy(), plan_o, 1e-2, "SO")
    _, fac = _gpu_factor(ctx, p, 6, 1, 1e-2, "SO")
    x = rhs(p.n, nrhs, 12)
    y_ref = ospand.apply(F, x)
    dx = _dev(x)
    dy = torch.zeros_like(dx)
    ctx.apply(fac, nrhs, dx, dy)
    y = dy.cpu().numpy().reshape(p.n, nrhs, order="F")
    for j in range(nrhs):
        assert np.linalg.norm(y[:, j] - y_ref[:, j]) <= 1e-11 * np.linalg.norm(y_ref[:, j]), j


@gpu
@pytest.mark.parametrize("scheme", ["FO", "SO"])
@pytest.mark.parametrize("name,make,depth,skip,eps,tol,nrhs", [
    ("lap2d_64", lambda: laplacian_2d(64), 6, 4, 1e-2, 1e-12, 1),
    ("lap3d_16", lambda: laplacian_3d(16), 6, 1, 1e-2, 1e-10, 4),
    ("fv3d_12", lambda: fv_diffusion_3d(12, 3.0, 1002), 5, 0, 1e-2, 1e-10, 2),
], ids=["lap2d_64", "lap3d_16", "fv3d_12"])
def test_pcg_matches_oracle(ctx, name, make, depth, skip, eps, tol, nrhs, scheme):
    p = make()
    print(f"pcg {name} {scheme}", flush=True)
    A = p.scipy()
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(A, plan_o, eps, scheme)
    b = rhs(p.n, nrhs, 2000)
    X, its, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
    _, fac = _gpu_factor(ctx, p, depth, skip, eps, scheme)
    db = _dev(b)
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, nrhs, db, dx, tol, 1000)
    x = dx.cpu().numpy().reshape(p.n, nrhs, order="F")
    for j in range(nrhs):
        assert abs(int(it[j]) - its[j]) <= 1
        assert rr[j] < 10 * tol
        assert np.linalg.norm(x[:, j] - X[:, j]) <= 1e-10 * np.linalg.norm(X[:, j])


@gpu
def test_eps_zero_is_exact_on_gpu(ctx):
    p = laplacian_3d(12)
    _, fac = _gpu_factor(ctx, p, 6, 0, 0.0, "SO")
    b = rhs(p.n, 1, 5)
    db = _dev(b)
    dy = torch.zeros_like(db)
    ctx.apply(fac, 1, db, dy)
    y = dy.cpu().numpy()
    res = np.linalg.norm(b[:, 0] - p.scipy() @ y) / np.linalg.norm(b)
    assert res < 1e-13
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, 1, db, dx, 1e-10, 100)
    assert it[0] == 1


@gpu
def test_not_spd_reports_step_and_cluster(ctx):
    from paper_2007_00789_amd import spand
    p = laplacian_2d(16)
    vals = p.vals.copy()
    v = 77
    diag = p.rowptr[v] + np.flatnonzero(p.colind[p.rowptr[v]:p.rowptr[v + 1]] == v)[0]
    vals[diag] = -4.0
    opts = spand.make_opts(depth=3, skip=0, eps=1e-2)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    with pytest.raises(spand.SpandError) as e:
        ctx.factor(plan, _dev(vals), opts)
    assert e.value.status == -3 and "step 3" in e.value.message


@gpu
def test_not_spd_in_a_step_without_sparsification(ctx):
    # steps 4 and 3 are not sparsified (skip 2): their breakdown flags are
    # read with those of step 2, and the failed block must still be named
    from paper_2007_00789_amd import spand
    p = laplacian_2d(32)
    vals = p.vals.copy()
    diag = p.rowptr[0] + np.flatnonzero(p.colind[p.rowptr[0]:p.rowptr[1]] == 0)[0]
    vals[diag] = -4.0
    opts = spand.make_opts(depth=4, skip=2, eps=1e-2)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    with pytest.raises(spand.SpandError) as e:
        ctx.factor(plan, _dev(vals), opts)
    assert e.value.status == -3 and "step 4" in e.value.message
    # the context stays usable: the unmodified matrix factors
    fac = ctx.factor(plan, _dev(p.vals), opts)
    fac.close()


@gpu
def test_not_spd_in_a_block_of_several_tiles(ctx):
    # A - 0.25 I on the 12^3 Laplacian (smallest eigenvalue 0.174): the leaf
    # interiors (300-432 rows) and the halves stay positive definite, the
    # Schur complement on the root separator (144 rows, three 64-row tiles)
    # does not.  The oracle fails on the same step and kind of block.
    from paper_2007_00789_amd import spand
    import scipy.sparse as sp
    p = laplacian_3d(12)
    A = (p.scipy() - 0.25 * sp.identity(p.n)).tocsr()
    A.sort_indices()
    assert np.array_equal(A.indptr, p.rowptr) and np.array_equal(A.indices, p.colind)
    with pytest.raises(ospand.NotSPD) as oe:
        ospand.factor(A, nd.analyze(p.rowptr, p.colind, p.coords, 2, 0), 1e-2, "SO")
    assert (oe.value.step, oe.value.what) == (1, "interface block")
    opts = spand.make_opts(depth=2, skip=0, eps=1e-2)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    with pytest.raises(spand.SpandError) as e:
        ctx.factor(plan, _dev(A.data), opts)
    assert e.value.status == -3
    assert f"interface block not SPD at step 1, cluster {oe.value.cluster}" in e.value.message
    # the unshifted matrix factors, and its large blocks are exact at eps = 0
    opts0 = spand.make_opts(depth=2, skip=0, eps=0.0)
    fac = ctx.factor(plan, _dev(p.vals), opts0)
    b = rhs(p.n, 1, 9)
    db = _dev(b)
    dy = torch.zeros_like(db)
    ctx.apply(fac, 1, db, dy)
    res = np.linalg.norm(b[:, 0] - p.scipy() @ dy.cpu().numpy()) / np.linalg.norm(b)
    assert res < 1e-13
    fac.close()


@gpu
def test_no_convergence_status(ctx):
    p = laplacian_2d(32)
    _, fac = _gpu_factor(ctx, p, 4, 0, 0.3, "FO")
    db = _dev(rhs(p.n, 1, 1))
    dx = torch.zeros_like(db)
    from paper_2007_00789_amd import spand
    with pytest.raises(spand.SpandError) as e:
        ctx.pcg(fac, 1, db, dx, 1e-14, 1)
    assert e.value.status == -4


@gpu
def test_factor_is_deterministic(ctx):
    p = fv_diffusion_3d(12, 3.0, 7)
    outs = []
    for _ in range(2):
        _, fac = _gpu_factor(ctx, p, 5, 0, 1e-2, "SO")
        db = _dev(rhs(p.n, 2, 3))
        dy = torch.zeros_like(db)
        ctx.apply(fac, 2, db, dy)
        outs.append(dy.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@gpu
def test_tiny_and_degenerate_problems(ctx):
    for p, depth in [(laplacian_2d(1), 2), (laplacian_2d(2), 3), (laplacian_2d(3, 1), 4)]:
        _, fac = _gpu_factor(ctx, p, depth, 0, 1e-2, "SO")
        b = rhs(p.n, 1, 2)
        db = _dev(b)
        dx = torch.zeros_like(db)
        it, rr = ctx.pcg(fac, 1, db, dx, 1e-12, 50)
        assert rr[0] < 1e-11


@gpu
@pytest.mark.parametrize("qr_group,qr_list_cap,xcd_local,one_launch", [
    (-1, -1, 1, 1), (1, -1, 1, 1), (3, -1, 1, 1), (5, 0, 1, 1), (8, 1, 1, 1), (3, -1, 0, 1),
    (8, 1, 0, 1), (32, -1, 1, 1), (32, -1, 1, 0), (5, 0, 1, 0)],
    ids=["single-wg", "lds-1", "lds-3", "lds-5-roundB", "lds-8-cap1", "lds-3-misplaced",
         "lds-8-cap1-misplaced", "lds-32", "lds-32-launch-per-round",
         "lds-5-roundB-launch-per-round"])
@pytest.mark.parametrize("name,make,depth,skip,eps", [CASES[1], CASES[3], CASES[4]],
                         ids=[CASES[1][0], CASES[3][0], CASES[4][0]])
def test_qr_paths_agree_with_oracle(ctx, name, make, depth, skip, eps, qr_group, qr_list_cap,
                                    xcd_local, one_launch):
    """Every QR path (single workgroup on a global workspace; cooperative groups
    of several workgroups with W in LDS, with and without the overflow round;
    groups reported as not placed on one XCD, which makes the factorization
    fall back to single-workgroup QRs; the rounds of co-resident groups of a
    colour in one launch, where each workgroup runs its groups one after the
    other, or one launch per round; groups of 32 workgroups give colours of
    several rounds on these problems) gives the oracle's (a, k, r, r2) and the
    same preconditioner."""
    p = make()
    print(f"qr paths {name} group={qr_group} cap={qr_list_cap} local={xcd_local} "
          f"one_launch={one_launch}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, "SO")
    _, fac = _gpu_factor(ctx, p, depth, skip, eps, "SO", qr_group=qr_group, qr_list_cap=qr_list_cap,
                         qr_xcd_local=xcd_local, qr_single_launch=one_launch)
    for l, recs in F.ranks.items():
        got = fac.ranks(l, plan_o.steps[l].n_clusters)
        for (p_, a, k, r, r2) in recs:
            assert (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2), (l, p_)
    x = rhs(p.n, 2, 13)
    y_ref = ospand.apply(F, x)
    dx = _dev(x)
    dy = torch.zeros_like(dx)
    ctx.apply(fac, 2, dx, dy)
    y = dy.cpu().numpy().reshape(p.n, 2, order="F")
    assert np.linalg.norm(y - y_ref) <= 1e-11 * np.linalg.norm(y_ref)


@gpu
def test_concurrent_contexts_keep_the_cooperative_qr(capfd):
    """Two contexts, each on its own stream, factoring at the same time from two
    threads (as the server's slots do): every cooperative QR group runs on its
    planned XCD (no fallback to the single-workgroup QR is reported) and both
    factors have the oracle's ranks."""
    import threading
    from paper_2007_00789_amd import spand
    p = laplacian_3d(16)
    depth, skip, eps = 6, 1, 1e-2
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, "SO")
    ctxs = [spand.Context(0) for _ in range(2)]
    results, errors = [[] for _ in ctxs], []

    def work(i):
        try:
            c = ctxs[i]
            opts = spand.make_opts(depth=depth, skip=skip, eps=eps, scheme="SO")
            plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, c)
            vals = _dev(p.vals)
            for _ in range(4):
                fac = c.factor(plan, vals, opts)
                results[i].append({l: fac.ranks(l, plan_o.steps[l].n_clusters) for l in F.ranks})
        except Exception as e:   # reported after the join
            errors.append(e)

    print("concurrent factorizations on two contexts", flush=True)
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for c in ctxs:
        c.close()
    assert not errors, errors
    err = capfd.readouterr().err
    assert "ran off" not in err, err
    for res in results:
        assert len(res) == 4
        for ranks in res:
            for l, recs in F.ranks.items():
                for (q, a, k, r, r2) in recs:
                    got = ranks[l]
                    assert (got["a"][q], got["k"][q], got["r"][q], got["r2"][q]) == (a, k, r, r2)


@gpu
def test_qr_rounds_in_one_launch_match_launch_per_round(ctx):
    """Groups of 32 workgroups on lap3d 16^3 need several rounds of co-resident
    groups per colour: in one launch (each workgroup runs its groups one after
    the other) the cooperative QR takes fewer launches than with one launch per
    round, and the factor is the same bit for bit (the apply of both)."""
    p = laplacian_3d(16)
    out = {}
    for one in (0, 1):
        print(f"qr rounds lap3d_16 group=32 one_launch={one}", flush=True)
        ctx.profile(True, only="k_cpqr_coop")
        _, fac = _gpu_factor(ctx, p, 6, 1, 1e-2, "SO", qr_group=32, qr_single_launch=one)
        launches = ctx.profile_entries()["k_cpqr_coop"][1]
        ctx.profile(False)
        dx = _dev(rhs(p.n, 2, 15))
        dy = torch.zeros_like(dx)
        ctx.apply(fac, 2, dx, dy)
        out[one] = (launches, dy.cpu().numpy())
    print(f"  k_cpqr_coop launches: per round {out[0][0]}, one launch per colour {out[1][0]}")
    assert out[1][0] < out[0][0]
    assert np.array_equal(out[0][1], out[1][1])


@gpu
@pytest.mark.parametrize("qr_group,lds_cols", [(1, 4), (3, 2), (5, 1), (0, 3), (2, 16)],
                         ids=["g1-lds4", "g3-lds2", "g5-lds1", "auto-lds3", "g2-lds16"])
@pytest.mark.parametrize("name,make,depth,skip,eps", [CASES[1], CASES[3], CASES[4]],
                         ids=[CASES[1][0], CASES[3][0], CASES[4][0]])
def test_qr_panel_columns_agree_with_oracle(ctx, name, make, depth, skip, eps, qr_group,
                                            lds_cols):
    """Cooperative QR workgroups that keep only some of their columns in LDS
    and the rest in place in the row panel (the path of interfaces wider than
    a group's LDS) give the oracle's ranks and the same preconditioner."""
    p = make()
    print(f"qr panel columns {name} group={qr_group} lds_cols={lds_cols}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, "SO")
    _, fac = _gpu_factor(ctx, p, depth, skip, eps, "SO", qr_group=qr_group, qr_lds_cols=lds_cols)
    for l, recs in F.ranks.items():
        got = fac.ranks(l, plan_o.steps[l].n_clusters)
        for (p_, a, k, r, r2) in recs:
            assert (got["k"][p_], got["r"][p_], got["r2"][p_]) == (k, r, r2), (l, p_)
    x = rhs(p.n, 2, 14)
    y_ref = ospand.apply(F, x)
    dx = _dev(x)
    dy = torch.zeros_like(dx)
    ctx.apply(fac, 2, dx, dy)
    y = dy.cpu().numpy().reshape(p.n, 2, order="F")
    assert np.linalg.norm(y - y_ref) <= 1e-11 * np.linalg.norm(y_ref)


# --- symmetric diagonal prescaling and coordinate-free analysis --------------

def _row_scaled_vals(p, seed):
    """values of S A S (S = diag(10^U[-3, 3])) in A's CSR order: a_ij (s_i s_j)"""
    s = 10.0 ** np.random.default_rng(seed).uniform(-3, 3, p.n)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    return p.vals * (s[rows] * s[p.colind])


def _csr(p, vals):
    import scipy.sparse as sp_
    return sp_.csr_matrix((vals, p.colind, p.rowptr), shape=(p.n, p.n))


@gpu
@pytest.mark.parametrize("coords_given", [True, False], ids=["geometric", "coordinate_free"])
@pytest.mark.parametrize("prescale", [1, 0])
def test_prescale_and_coordinate_free_match_oracle(ctx, prescale, coords_given):
    from paper_2007_00789_amd import spand
    p = fv_diffusion_3d(10, 2.0, 1003)
    depth, skip, eps, nrhs, tol = 5, 1, 1e-2, 2, 1e-10
    print(f"prescale {prescale} coords {coords_given}", flush=True)
    vals = _row_scaled_vals(p, 77) if prescale else p.vals
    A = _csr(p, vals)
    coords = p.coords if coords_given else None
    plan_o = nd.analyze(p.rowptr, p.colind, coords, depth, skip)
    F = ospand.factor(A, plan_o, eps, "SO", prescaled=bool(prescale))
    opts = spand.make_opts(depth=depth, skip=skip, eps=eps, scheme="SO", prescale=prescale)
    plan = spand.analyze(p.n, p.rowptr, p.colind, coords, opts, ctx)
    fac = ctx.factor(plan, _dev(vals), opts)
    ref = _oracle_ranks(F)
    for l in range(depth, 0, -1):
        st = plan_o.steps[l]
        if not st.sparsified:
            continue
        got = fac.ranks(l, st.n_clusters)
        for p_, (a, k, r, r2) in ref[l].items():
            assert (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2), \
                (l, p_)
    b = rhs(p.n, nrhs, 2100)
    X, its, _ = opcg.pcg_multi(lambda v: A @ v, lambda v: ospand.apply(F, v), b, tol)
    db = _dev(b)
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, nrhs, db, dx, tol, 1000)
    x = dx.cpu().numpy().reshape(p.n, nrhs, order="F")
    for j in range(nrhs):
        assert abs(int(it[j]) - its[j]) <= 1
        assert rr[j] < 10 * tol
        assert np.linalg.norm(x[:, j] - X[:, j]) <= 1e-10 * np.linalg.norm(X[:, j])
    # the apply alone: y = D M~ D b
    dy = torch.zeros_like(db)
    ctx.apply(fac, nrhs, db, dy)
    Y = ospand.apply(F, b)
    y = dy.cpu().numpy().reshape(p.n, nrhs, order="F")
    assert np.linalg.norm(y - Y) <= 1e-10 * np.linalg.norm(Y)
    fac.close()


@gpu
def test_prescale_rejects_a_nonpositive_diagonal(ctx):
    from paper_2007_00789_amd import spand
    p = laplacian_2d(16)
    vals = p.vals.copy()
    v = 40
    diag = p.rowptr[v] + np.flatnonzero(p.colind[p.rowptr[v]:p.rowptr[v + 1]] == v)[0]
    vals[diag] = 0.0
    opts = spand.make_opts(depth=3, skip=0, eps=1e-2, prescale=1)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    with pytest.raises(spand.SpandError) as e:
        ctx.factor(plan, _dev(vals), opts)
    assert e.value.status == -3 and "row 40" in e.value.message


@gpu
@pytest.mark.parametrize("scheme", ["FO", "SO"])
def test_high_contrast_field_of_table1(ctx, scheme):
    """The rho = 100 high-contrast field of the Table 1 study (Sec. 4.1: uniform
    noise, Gaussian blur sigma = 2, quantised to rho^{+-1}), 192 x 192, depth
    round(log2(n/64)) = 9, skip 4, b = ones as in the paper, eps 1e-2: every
    interface goes through the cooperative QR; ranks (a, k, r, r2) bit-exact,
    n_cg +-1 and the solution within 1e-10 relative of the oracle's."""
    d, rho = 192, 100.0
    p = high_contrast_2d(d, rho, seed=5000 + d)
    depth = int(round(np.log2(p.n / 64.0)))
    print(f"high contrast rho={rho:g} d={d} {scheme}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, 4)
    A = p.scipy()
    F = ospand.factor(A, plan_o, 1e-2, scheme)
    _, fac = _gpu_factor(ctx, p, depth, 4, 1e-2, scheme)
    nsp = 0
    for l, recs in F.ranks.items():
        got = fac.ranks(l, plan_o.steps[l].n_clusters)
        for (p_, a, k, r, r2) in recs:
            assert (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2), (l, p_)
            nsp += 1
    assert nsp > 50
    b = np.ones(p.n)
    x_ref, it_ref, _ = opcg.pcg(lambda v: A @ v, lambda v: ospand.apply(F, v), b, 1e-10)
    db = _dev(b)
    dx = torch.zeros_like(db)
    it, rr = ctx.pcg(fac, 1, db, dx, 1e-10, 1000)
    x = dx.cpu().numpy()
    assert abs(int(it[0]) - it_ref) <= 1, (int(it[0]), it_ref)
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


@gpu
def test_apply_graph_replays_match_plain_launches(ctx):
    """opts.apply_graph = 1: the apply captured in a HIP graph at its first use
    and replayed afterwards gives, on every replay, exactly what the plain
    launches give (same kernels, same order), with eager work and
    synchronizations between the replays; PCG likewise."""
    from paper_2007_00789_amd import spand
    p = laplacian_3d(16)
    print("apply graph replays", flush=True)
    res = {}
    for g in (0, 1):
        opts = spand.make_opts(depth=6, skip=1, eps=1e-2, scheme="SO", apply_graph=g)
        plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
        res[g] = (plan, ctx.factor(plan, _dev(p.vals), opts))
    x = _dev(rhs(p.n, 3, 41))
    yg = torch.zeros_like(x)
    yp = torch.zeros_like(x)
    for rep in range(4):
        ctx.apply(res[1][1], 3, x, yg)          # capture at rep 0, replays after
        torch.cuda.synchronize()
        ctx.apply(res[0][1], 3, x, yp)          # plain launches in between
        x.mul_(1.0 + 0.25 * rep)                # eager work on the captured input buffer
        torch.cuda.synchronize()
        assert torch.equal(yg, yp), rep
    b = _dev(rhs(p.n, 2, 42))
    xs = {g: torch.zeros_like(b) for g in (0, 1)}
    its = {g: ctx.pcg(res[g][1], 2, b, xs[g], 1e-10, 1000) for g in (0, 1)}
    assert np.array_equal(its[0][0], its[1][0])
    assert torch.equal(xs[0], xs[1])


@gpu
@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("name,make,depth,skip,eps", [CASES[1], CASES[3], CASES[5]],
                         ids=[CASES[1][0], CASES[3][0], CASES[5][0]])
def test_gemm_tiles_agree_with_oracle(ctx, name, make, depth, skip, eps, tile):
    """Both GEMM kernels (64 x 64 tiles; 128 x 128 tiles with double-buffered
    k-slabs) for every GEMM launch: ranks (a, k, r, r2) bit-exact and the
    apply within 1e-11 of the oracle's."""
    from paper_2007_00789_amd import spand
    p = make()
    print(f"gemm tile {tile} {name}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, "SO")
    opts = spand.make_opts(depth=depth, skip=skip, eps=eps, scheme="SO", gemm_tile=tile)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
    fac = ctx.factor(plan, _dev(p.vals), opts)
    for l, recs in F.ranks.items():
        got = fac.ranks(l, plan_o.steps[l].n_clusters)
        for (p_, a, k, r, r2) in recs:
            assert (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2), (l, p_)
    x = rhs(p.n, 2, 17)
    y_ref = ospand.apply(F, x)
    dx = _dev(x)
    dy = torch.zeros_like(dx)
    ctx.apply(fac, 2, dx, dy)
    y = dy.cpu().numpy().reshape(p.n, 2, order="F")
    assert np.linalg.norm(y - y_ref) <= 1e-11 * np.linalg.norm(y_ref)


@gpu
@pytest.mark.parametrize("name,make,depth,skip,eps", [CASES[3], CASES[4], CASES[5]],
                         ids=[CASES[3][0], CASES[4][0], CASES[5][0]])
def test_small_block_gemm_agrees_with_oracle(ctx, name, make, depth, skip, eps):
    """With the tile left to the library, GEMM blocks of at most 32 x 32 run on
    the one-wave-per-block kernel (the profile shows its launches): ranks
    (a, k, r, r2) bit-exact and the apply within 1e-11 of the oracle's, in FP64
    and (against the FP64 oracle, at the FP32 bar) in FP32."""
    from paper_2007_00789_amd import spand
    p = make()
    print(f"small-block gemm {name}", flush=True)
    plan_o = nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)
    F = ospand.factor(p.scipy(), plan_o, eps, "SO")
    x = rhs(p.n, 2, 19)
    y_ref = ospand.apply(F, x)
    for precision, bar in (("FP64", 1e-11), ("FP32", 1e-4)):
        opts = spand.make_opts(depth=depth, skip=skip, eps=eps, scheme="SO", precision=precision)
        plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
        ctx.profile(True)
        fac = ctx.factor(plan, _dev(p.vals), opts)
        torch.cuda.synchronize()
        prof = ctx.profile_entries()
        ctx.profile(False)
        assert prof.get("k_gemm_small", (0, 0, 0))[1] > 0, sorted(prof)
        ndiff = 0   # interfaces whose (a, k, r, r2) differ from the FP64 oracle's
        for l, recs in F.ranks.items():
            got = fac.ranks(l, plan_o.steps[l].n_clusters)
            for (p_, a, k, r, r2) in recs:
                same = (got["a"][p_], got["k"][p_], got["r"][p_], got["r2"][p_]) == (a, k, r, r2)
                if precision == "FP64":
                    assert same, (l, p_)
                ndiff += not same
        dx = _dev(x)
        dy = torch.zeros_like(dx)
        ctx.apply(fac, 2, dx, dy)
        y = dy.cpu().numpy().reshape(p.n, 2, order="F")
        err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        print(f"  {precision}: apply error {err:.2e}, small-kernel launches {prof['k_gemm_small'][1]}, "
              f"QR launches {prof.get('k_cpqr_coop', (0, 0, 0))[1]} cooperative + "
              f"{prof.get('k_cpqr', (0, 0, 0))[1]} single-workgroup, interfaces with other ranks "
              f"than the FP64 oracle {ndiff}", flush=True)
        assert err <= bar, (precision, err)
