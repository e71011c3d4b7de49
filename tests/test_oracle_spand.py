"""Pins of the oracle's factorization, apply and PCG against what the paper
and the mathematics fix:

* eps = 0 is the exact block Cholesky in nested-dissection order (Sec. 3.2);
  with no sparsified level the factor equals numpy's Cholesky of P A P^T.
* Props. 1, 2 and 3 (Sec. 2.3): the spectrum of the two-level preconditioned
  matrix equals the closed forms built from s = ||Lhat^{-1} Ehat^T||.
* The full second-order scheme only drops the negative semidefinite -E^T E,
  so L L^T >= A and every eigenvalue of L^{-1} A L^{-T} lies in (0, 1]
  (Sec. 2.2 "implicit Schur compensation", Prop. 2); the first-order scheme
  has eigenvalues above 1.
* ||I - L^{-1} A L^{-T}||_2 decays like eps (first order) and eps^2 (second
  order), by dense brute force on a small grid (Secs. 2.1, 2.2).
* Theorem 1 (Sec. 2.3.5): CG residuals satisfy r1_{2k} = r2_k when C^T b1 = 0.
* PCG converges to the sparse direct solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d, rhs
from oracle import nd, spand, pcg
from oracle.nd import Plan, Step


def _plan(p, depth, skip=4):
    return nd.analyze(p.rowptr, p.colind, p.coords, depth, skip)


def _precond_matrix(F, A):
    Li = spand.dense_Linv(F)
    S = Li @ A @ Li.T
    return (S + S.T) / 2


@pytest.mark.parametrize("make,depth,skip", [
    (lambda: laplacian_2d(24), 4, 0),
    (lambda: laplacian_3d(8), 5, 0),
    (lambda: fv_diffusion_3d(7, 3.0, 11), 4, 0),
])
@pytest.mark.parametrize("scheme", ["FO", "SO", "SF"])
def test_eps_zero_is_exact(make, depth, skip, scheme):
    p = make()
    A = p.scipy()
    F = spand.factor(A, _plan(p, depth, skip), 0.0, scheme)
    Ad = A.toarray()
    S = _precond_matrix(F, Ad)
    assert np.linalg.norm(np.eye(p.n) - S, 2) < 1e-11
    b = rhs(p.n, 1, 7)[:, 0]
    x = spand.apply(F, b)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-13
    _, it, _ = pcg.pcg(lambda v: A @ v, lambda v: spand.apply(F, v), b, 1e-10)
    assert it == 1


def test_no_sparsification_equals_dense_cholesky():
    p = laplacian_3d(6)
    A = p.scipy()
    D = 4
    F = spand.factor(A, _plan(p, D, skip=D), 0.3, "SO")
    assert not any(op[0] == "sparsify" for op in F.ops)
    order = np.concatenate([op[1] for op in F.ops if op[0] == "interior"])
    assert np.array_equal(np.sort(order), np.arange(p.n))
    Ad = A.toarray()[np.ix_(order, order)]
    Lref = np.linalg.cholesky(Ad)
    where = np.empty(p.n, dtype=np.int64)
    where[order] = np.arange(p.n)
    Lmine = np.zeros_like(Lref)
    for op in F.ops:
        _, ps, L, nbrs = op
        Lmine[np.ix_(where[ps], where[ps])] = L
        for pw, G in nbrs:
            Lmine[np.ix_(where[pw], where[ps])] = G.T
    assert np.allclose(Lmine, Lref, atol=1e-12)


def test_second_order_spectrum_in_unit_interval_first_order_above():
    p = laplacian_2d(20)
    A = p.scipy().toarray()
    plan = _plan(p, 4, 0)
    for eps in [0.3, 0.1, 0.03]:
        ev2 = np.linalg.eigvalsh(_precond_matrix(spand.factor(A, plan, eps, "SO"), A))
        assert ev2.min() > 0 and ev2.max() <= 1 + 1e-12
        ev1 = np.linalg.eigvalsh(_precond_matrix(spand.factor(A, plan, eps, "FO"), A))
        assert ev1.min() > 0 and ev1.max() > 1 + 1e-6


def test_schemes_share_ranks_and_trailing_matrix():
    p = laplacian_3d(10)
    A = p.scipy()
    plan = _plan(p, 6, 1)
    fs = {s: spand.factor(A, plan, 1e-2, s) for s in ("FO", "SO", "SF")}
    assert spand.all_ranks(fs["FO"]) == spand.all_ranks(fs["SO"])
    assert [r[:5] for r in spand.all_ranks(fs["SF"])] == [r[:5] for r in spand.all_ranks(fs["FO"])]
    # identical elimination blocks on every level (bit for bit)
    for a, b in zip(fs["FO"].ops, fs["SO"].ops):
        assert a[0] == b[0]
        if a[0] == "interior":
            assert np.array_equal(a[2], b[2])
    assert fs["SO"].nnz_L > fs["SF"].nnz_L >= fs["FO"].nnz_L


@pytest.mark.slow
def test_eps_slopes_brute_force():
    p = laplacian_2d(32)
    A = p.scipy().toarray()
    plan = _plan(p, 5, 0)
    epss = np.array([1e-1, 3e-2, 1e-2, 3e-3, 1e-3])
    slopes = {}
    for scheme in ("FO", "SO"):
        err = [np.linalg.norm(np.eye(p.n) - _precond_matrix(spand.factor(A, plan, e, scheme), A), 2)
               for e in epss]
        slopes[scheme] = np.polyfit(np.log(epss), np.log(err), 1)[0]
    # ranks move in discrete jumps, so the slopes are bands around 1 and 2
    # (measured: 1.18 and 2.36)
    assert 0.7 <= slopes["FO"] <= 1.3, slopes
    assert 1.6 <= slopes["SO"] <= 2.4, slopes
    assert slopes["SO"] > slopes["FO"] + 0.7


def _two_level(n1=14, n2=30, n3=9, seed=0):
    """A = M M^T with M block lower bidiagonal: A13 = 0, and A12 = M11 M21^T
    with geometrically decaying singular values."""
    rng = np.random.default_rng(seed)
    n = n1 + n2 + n3
    M = np.zeros((n, n))
    i1, i2, i3 = slice(0, n1), slice(n1, n1 + n2), slice(n1 + n2, n)
    M[i1, i1] = np.eye(n1) + 0.3 * np.tril(rng.standard_normal((n1, n1)), -1)
    M[i2, i2] = np.eye(n2) + 0.3 * np.tril(rng.standard_normal((n2, n2)), -1)
    M[i3, i3] = np.eye(n3) + 0.3 * np.tril(rng.standard_normal((n3, n3)), -1)
    U, _ = np.linalg.qr(rng.standard_normal((n2, n2)))
    V, _ = np.linalg.qr(rng.standard_normal((n1, n1)))
    k = min(n1, n2)
    M[i2, i1] = 0.8 * U[:, :k] @ np.diag(0.5 ** np.arange(k)) @ V[:, :k].T
    M[i3, i2] = 0.5 * rng.standard_normal((n3, n2))
    return M @ M.T, (n1, n2, n3)


def _two_level_plan(sizes):
    n1, n2, n3 = sizes
    idx = np.arange(n1 + n2 + n3)
    verts = [idx[:n1], idx[n1:n1 + n2], idx[n1 + n2:]]
    adj = [np.array([0, 1]), np.array([0, 1, 2]), np.array([1, 2])]
    s1 = Step(1, [(1, 0, 0), (1, 0, 1), (1, 0, 2)], 0, adj, np.array([0, 1, 0]), True, [0],
              None, verts)
    s0 = Step(0, [(0, 0, 0)], 1, [np.array([0])], np.array([-1]), False, [], [[0, 1, 2]], None)
    return Plan(n1 + n2 + n3, 1, 0, np.zeros(0), np.zeros(0), idx, [], {1: s1, 0: s0})


@pytest.mark.parametrize("eps", [0.2, 0.05, 0.01])
def test_props_1_2_3_two_level(eps):
    A, sizes = _two_level()
    n1, n2, n3 = sizes
    n = sum(sizes)
    plan = _two_level_plan(sizes)
    # the two-level construction, independently of the oracle (scipy's pivoted QR)
    i1, i2, i3 = slice(0, n1), slice(n1, n1 + n2), slice(n1 + n2, n)
    Z = sla.block_diag(*[np.linalg.cholesky(A[i, i]) for i in (i1, i2, i3)])
    At = sla.solve_triangular(Z, sla.solve_triangular(Z, A, lower=True).T, lower=True).T
    W = At[i1, i2]
    Q, R, _ = sla.qr(W, pivoting=True)
    d = np.abs(np.diag(R))
    r = int(np.sum(np.cumprod(d >= eps * d[0])))
    r2 = int(np.sum(np.cumprod(d >= eps * eps * d[0])))
    Qc, Qf = Q[:, :r], Q[:, r:]
    E = Qf.T @ W
    m = r + n2 + n3
    Ahat = np.zeros((m, m))
    Ahat[:r, :r] = np.eye(r)
    Ahat[:r, r:r + n2] = Qc.T @ W
    Ahat[r:r + n2, :r] = (Qc.T @ W).T
    Ahat[r:, r:] = At[n1:, n1:]
    Lh = np.linalg.cholesky(Ahat)
    Ehat = np.zeros((n1 - r, m))
    Ehat[:, r:r + n2] = E
    C = sla.solve_triangular(Lh, Ehat.T, lower=True)       # Lhat^{-1} Ehat^T
    s = np.linalg.norm(C, 2)
    f = n1 - r
    # Prop. 1: [[I, C^T], [C, I]]
    P1 = np.eye(f + m)
    P1[:f, f:] = C.T
    P1[f:, :f] = C
    # Prop. 2: diag(I, I - C C^T)
    P2 = np.eye(f + m)
    P2[f:, f:] -= C @ C.T
    # Prop. 3 with f = (f1, f2): f2 = pivots r..r2-1
    E1 = Q[:, r2:].T @ W
    E2 = Q[:, r:r2].T @ W
    C1 = np.zeros((m, n1 - r2))
    C2 = np.zeros((m, r2 - r))
    C1 = sla.solve_triangular(Lh, np.vstack([np.zeros((r, n1 - r2)), E1.T, np.zeros((n3, n1 - r2))]), lower=True)
    C2 = sla.solve_triangular(Lh, np.vstack([np.zeros((r, r2 - r)), E2.T, np.zeros((n3, r2 - r))]), lower=True)
    f1 = n1 - r2
    P3 = np.eye(f + m)
    P3[:f1, f:] = C1.T
    P3[f:, :f1] = C1
    P3[f:, f:] -= C2 @ C2.T

    got = {}
    for scheme in ("FO", "SO", "SF"):
        F = spand.factor(A, plan, eps, scheme)
        assert [rk[3] for rk in F.ranks[1]] == [r]
        got[scheme] = np.linalg.eigvalsh(_precond_matrix(F, A))
    assert np.allclose(got["FO"], np.linalg.eigvalsh(P1), atol=1e-10)
    assert np.allclose(got["SO"], np.linalg.eigvalsh(P2), atol=1e-10)
    assert np.allclose(got["SF"], np.linalg.eigvalsh(P3), atol=1e-10)
    k1 = got["FO"].max() / got["FO"].min()
    k2 = got["SO"].max() / got["SO"].min()
    assert k1 == pytest.approx((1 + s) / (1 - s), rel=1e-9)     # eq. cond-1
    assert k2 == pytest.approx(1 / (1 - s * s), rel=1e-9)       # eq. cond-2


def test_theorem_1_residuals():
    rng = np.random.default_rng(4)
    n1, n2 = 14, 8
    C = rng.standard_normal((n1, n2))
    C *= 0.9 / np.linalg.norm(C, 2)
    U, _, _ = np.linalg.svd(C)
    b1 = U[:, n2:] @ rng.standard_normal(n1 - n2)         # C^T b1 = 0
    b = np.concatenate([b1, rng.standard_normal(n2)])
    A1 = np.block([[np.eye(n1), C], [C.T, np.eye(n2)]])
    A2 = np.block([[np.eye(n1), np.zeros((n1, n2))], [np.zeros((n2, n1)), np.eye(n2) - C.T @ C]])
    ident = lambda v: v.copy()
    _, _, h1 = pcg.pcg(lambda v: A1 @ v, ident, b, 1e-300, 10)
    _, _, h2 = pcg.pcg(lambda v: A2 @ v, ident, b, 1e-300, 5)
    for k in range(1, 6):
        assert h1[2 * k] == pytest.approx(h2[k], rel=1e-7, abs=1e-13)
    # and the statement is not vacuous: odd first-order steps differ
    assert abs(h1[1] - h2[1]) > 1e-3


def test_pcg_matches_direct_solve_and_second_order_halves():
    p = laplacian_2d(64)
    A = p.scipy()
    plan = _plan(p, 6)
    b = rhs(p.n, 1, 2000)[:, 0]
    xd = spla.spsolve(sp.csc_matrix(A), b)
    its = {}
    for scheme in ("FO", "SO"):
        F = spand.factor(A, plan, 1e-2, scheme)
        x, its[scheme], _ = pcg.pcg(lambda v: A @ v, lambda v: spand.apply(F, v), b, 1e-12)
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-12
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
    assert its["SO"] < its["FO"]


def test_not_spd_is_reported():
    p = laplacian_2d(10)
    A = p.scipy().tolil()
    A[37, 37] = -4.0
    with pytest.raises(spand.NotSPD) as ei:
        spand.factor(A.tocsr(), _plan(p, 3), 1e-2, "SO")
    assert ei.value.step == 3


@pytest.mark.parametrize("eps", [0.5, 0.1, 1e-2])
def test_high_contrast_stays_spd(eps):
    p = fv_diffusion_3d(8, 3.0, 1002)
    A = p.scipy()
    plan = _plan(p, 5, 1)
    for scheme in ("FO", "SO", "SF"):
        F = spand.factor(A, plan, eps, scheme)       # raises NotSPD otherwise
        ev = np.linalg.eigvalsh(_precond_matrix(F, A.toarray()))
        assert ev.min() > 0
        if scheme == "SO":
            assert ev.max() <= 1 + 1e-10


def test_nnz_counts_match_the_stored_factor():
    p = laplacian_3d(8)
    A = p.scipy()
    F = spand.factor(A, _plan(p, 5, 1), 1e-2, "SO")
    cnt = 0
    for op in F.ops:
        if op[0] == "interior":
            ns = op[1].size
            cnt += ns * (ns + 1) // 2 + sum(G.size for _, G in op[3])
        elif op[0] == "scale":
            a = op[1].size
            cnt += a * (a + 1) // 2
        else:
            _, pp, V, taus, (f0, f1), nbr_pos, E = op
            cnt += sum(v.size for v in V) + len(taus)
            if E is not None and E.size:
                piv_cols = np.abs(E).sum(axis=0) == 0
                assert piv_cols.sum() >= f0          # E = [0 R_ff] P^T
                cnt += E.shape[0] * (E.shape[1] - f0)
    assert cnt == F.nnz_L
    assert spand.mu(F, A) == F.nnz_L / p.nnz


# --- symmetric diagonal prescaling -----------------------------------------

def _row_scaled(p, seed):
    """S A S with S = diag(10^U[-3, 3]): same spectrum structure, wild diagonal."""
    import scipy.sparse as sp_
    s = 10.0 ** np.random.default_rng(seed).uniform(-3, 3, p.n)
    C = p.scipy().tocoo()
    return sp_.csr_matrix((C.data * (s[C.row] * s[C.col]), (C.row, C.col)), shape=C.shape)


def test_prescale_unit_diagonal_and_errors():
    p = fv_diffusion_3d(6, 2.0, 11)
    As, d = spand.prescale(_row_scaled(p, 3))
    assert np.allclose(As.diagonal(), 1.0, rtol=4e-16 * 4, atol=0)
    assert abs(As - As.T).max() == 0.0          # a_ij (d_i d_j): exactly symmetric
    A = p.scipy().tolil()
    A[5, 5] = 0.0
    with pytest.raises(spand.NotSPD) as e:
        spand.prescale(A.tocsr())
    assert e.value.cluster == 5


def test_prescaled_factor_is_exact_at_eps0():
    # eps = 0 keeps every reflector, so D M~ D = (D^{-1} (D A D)^{-1} D^{-1})... = A^{-1}
    p = fv_diffusion_3d(6, 2.0, 12)
    A = _row_scaled(p, 4)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 3, 0)
    F = spand.factor(A, plan, 0.0, "SO", prescaled=True)
    X = np.random.default_rng(5).standard_normal((p.n, 2))
    Y = spand.apply(F, A @ X)
    assert np.linalg.norm(Y - X) <= 1e-9 * np.linalg.norm(X)


def test_prescaling_removes_a_diagonal_scaling():
    # D' of S A S is S^{-1} D, so the prescaled operator D' S A S D' is D A D up
    # to rounding: the same ranks and iteration counts as for A itself
    p = fv_diffusion_3d(8, 2.0, 13)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 4, 0)
    A, As = p.scipy(), _row_scaled(p, 6)
    Fa = spand.factor(A, plan, 1e-2, "SO", prescaled=True)
    Fs = spand.factor(As, plan, 1e-2, "SO", prescaled=True)
    Fn = spand.factor(As, plan, 1e-2, "SO")
    b = np.ones(p.n)
    _, it_a, _ = pcg.pcg(lambda v: A @ v, lambda v: spand.apply(Fa, v), b, 1e-10)
    _, it_s, _ = pcg.pcg(lambda v: As @ v, lambda v: spand.apply(Fs, v), b, 1e-10)
    _, it_n, _ = pcg.pcg(lambda v: As @ v, lambda v: spand.apply(Fn, v), b, 1e-10, maxit=400)
    assert abs(it_a - it_s) <= 1
    assert it_n >= it_s


def test_flop_counter_hand_count_grid():
    """The algorithmic flop counter on an 8 x 8 grid, depth 2, skip 0, eps 0,
    against a count made by hand from the partition rule: leaves LL 3x3, LR
    3x4, RL 4x3, RR 4x4 (n = 9, 12, 12, 16 with k = 7, 7, 8, 8); step-2
    interfaces S1L (a 3, k 8), S1R (4, 8), S0a and S0b (4, 11) kept whole at
    eps = 0 (r = a); step-1 interiors S1L, S1R (k 8) and the interface S0
    (a 8, no coupling left: k = 0, r = 0).  Per unit: interior n^3/3 + n^2 k +
    n k^2, scaling a^3/3 + a^2 k, pivoted QR sum_{j<r} 4 (a-j)(k-j)."""
    from synthetic import laplacian_2d
    p = laplacian_2d(8)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 2, 0)
    F = spand.factor(p.scipy(), plan, 0.0, "SO")
    step2 = (243 + 567 + 441) + (576 + 1008 + 588) + (576 + 1152 + 768) + (4096 / 3 + 2048 + 1024)
    step2 += (9 + 72) + (64 / 3 + 128) + 2 * (64 / 3 + 176)                 # scaling
    step2 += (96 + 56 + 24) + (128 + 84 + 48 + 20) + 2 * (176 + 120 + 72 + 32)   # QR
    step1 = (9 + 72 + 192) + (64 / 3 + 128 + 256) + 512 / 3
    assert F.flops[2] == pytest.approx(step2, rel=1e-14)
    assert F.flops[1] == pytest.approx(step1, rel=1e-14)
    assert F.flops[0] == 0.0
    assert sum(F.flops.values()) == pytest.approx(13086 + 1 / 3, rel=1e-14)


@pytest.mark.parametrize("scheme", ["FO", "SO", "SF"])
def test_flop_counter_hand_count_two_level(scheme):
    """The counter on the two-level construction (interfaces of 14, 30 and 9
    variables, no interiors; the plan sparsifies interface 0 only): every
    interface of the step is scaled (a^3/3 each); the sparsified one adds
    a^2 k + sum_{j<nref} 4 (a-j)(k-j) with k its coupling width when it is
    sparsified (30: interface 1 is still whole), nref = r (FO, SO) or r2 (SF);
    the root is the Cholesky of the 5 + 30 + 9 coarse variables left.  The
    rank comes from the factor; the widths and terms are counted here."""
    A, sizes = _two_level()
    n1, n2, n3 = sizes
    F = spand.factor(A, _two_level_plan(sizes), 0.05, scheme)
    [(c, a, k, r, r2)] = F.ranks[1]
    assert (c, a, k) == (0, n1, n2)
    nref = r2 if scheme == "SF" else r
    qr = sum(4.0 * (n1 - j) * (n2 - j) for j in range(nref))
    step1 = n1 ** 3 / 3 + n2 ** 3 / 3 + n3 ** 3 / 3 + n1 * n1 * n2 + qr
    assert F.flops[1] == pytest.approx(step1, rel=1e-14)
    assert F.flops[0] == pytest.approx((r + n2 + n3) ** 3 / 3, rel=1e-14)
