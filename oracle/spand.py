"""The spaND factorization (Alg. 2), its apply and its counters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State.  Every cluster of a step has a list of positions into an n-vector in
the original vertex numbering (its current variables) and a dense block
B[i, j] for every adjacent pair, held in both orientations.

Step l, in the paper's order (Alg. 2; Sec. 1 for the block elimination,
eq. prescale for the scaling, Alg. 1 and Sec. 2 for the sparsification):

(a) every interior s, in canonical order: L_s = chol(B_ss); for each neighbour
    w, G_w = L_s^{-1} B_sw (so F_ws = B_ws L_s^{-T} = G_w^T); then
    B_{w1 w2} -= G_w1^T G_w2 for every neighbour pair, w1 = w2 included.
    G_s of Alg. 2 is read as [[L_s^{-1}, 0], [-B_ws B_ss^{-1}, I]]: the printed
    (2,1) block -A_ws L_s^{-T} does not satisfy G A G^T = diag(I, S), the form
    used here does.
(b) sparsified steps only: Z_p = chol(B_pp) for every interface, then every
    block is scaled on both sides, B_pq <- Z_p^{-1} B_pq Z_q^{-T}, and B_pp <- I
    (block-Jacobi / double-sided scaling, Sec. 2.3.2).
(c) sparsified steps only, interfaces in (colour, canonical) order:
    W = [B_{p,w1} ... B_{p,wm}] (neighbours in canonical order), Y = Q^T W from
    the early-stopping CPQR (oracle.dense), B_{p,w} <- Y[:r, cols of w],
    B_pp <- I_r, and the interface keeps its first r positions (coarse); the
    fine variables are final.  The trailing matrix is the same for every scheme
    (eq. trailing-1/-2/-3); only the stored term differs:
      first order       : nothing,
      full second order : E = Q_f^T W = Y[r:]        (eq. trailing-2),
      superfine         : E_2 = Q_f2^T W = Y[r:r2]   (eq. trailing-3, eq. rrqr),
                          with Q built from r2 reflectors (eps^2 rank).
(d) merge: each step-(l-1) cluster concatenates the current positions of its
    children; its blocks are assembled from the children's blocks (zero where
    the children were not adjacent).

The recorded operations give L^{-1} = B_0 B_1 ... B_D (apply B_D first); the
preconditioner is M = L^{-T} L^{-1} (Alg. 2 caption).

Prescaling (optional; the experiments scale A symmetrically by its diagonal,
Sec. 4): with d = diag(A)^{-1/2} the factorization runs on D A D, entry
(i, j) = a_ij (d_i d_j) (exactly symmetric), and the preconditioner of A is
D M~ D, M~ the one of D A D.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .dense import cpqr, apply_qt, apply_q

FIRST_ORDER, SECOND_ORDER, SUPERFINE = "FO", "SO", "SF"


class NotSPD(Exception):
    def __init__(self, step, cluster, what):
        super().__init__(f"{what} not SPD at step {step}, cluster {cluster}")
        self.step, self.cluster, self.what = step, cluster, what


@dataclass
class Factor:
    n: int
    scheme: str
    eps: float
    ops: list = field(default_factory=list)
    ranks: dict = field(default_factory=dict)      # l -> list of (cluster, a, k, r, r2)
    shapes: dict = field(default_factory=dict)     # l -> list of (cluster, n_s, k_s)
    nnz_L: int = 0
    flops: dict = field(default_factory=dict)      # l -> algorithmic flops of the step
    root_size: int = 0
    dscale: np.ndarray | None = None               # prescaling: diag(A)^{-1/2}


def _chol(B, step, c, what):
    if B.shape[0] == 0:
        return np.zeros((0, 0))
    try:
        return np.linalg.cholesky(B)
    except np.linalg.LinAlgError:
        raise NotSPD(step, c, what) from None


def _lsolve(L, X):
    return sla.solve_triangular(L, X, lower=True) if L.shape[0] else X.copy()


def _ltsolve(L, X):
    return sla.solve_triangular(L, X, lower=True, trans="T") if L.shape[0] else X.copy()


def _assemble_leaf_blocks(A, st):
    """B[i, j] = A[vars_i, vars_j] for every adjacent pair of the first step."""
    n = A.shape[0]
    nc = st.n_clusters
    cid = np.empty(n, dtype=np.int64)
    loc = np.empty(n, dtype=np.int64)
    for c, vs in enumerate(st.verts):
        cid[vs] = c
        loc[vs] = np.arange(vs.size)
    B = {}
    for i in range(nc):
        for j in st.adj[i]:
            B[(i, int(j))] = np.zeros((st.verts[i].size, st.verts[int(j)].size))
    coo = A.tocoo()
    code = cid[coo.row] * nc + cid[coo.col]
    order = np.argsort(code, kind="stable")
    code, r, c, v = code[order], coo.row[order], coo.col[order], coo.data[order]
    bounds = np.flatnonzero(np.diff(code)) + 1
    for seg in np.split(np.arange(code.size), bounds):
        if seg.size == 0:
            continue
        key = (int(code[seg[0]] // nc), int(code[seg[0]] % nc))
        B[key][loc[r[seg]], loc[c[seg]]] = v[seg]
    return B


def prescale(A):
    """(D A D, d) with d = diag(A)^{-1/2}; NotSPD(-1, row) on a non-positive diagonal."""
    A = sp.csr_matrix(A)
    a = A.diagonal()
    bad = np.flatnonzero(~(a > 0.0))
    if bad.size:
        raise NotSPD(-1, int(bad[0]), "prescale diagonal")
    d = 1.0 / np.sqrt(a)
    C = A.tocoo()
    As = sp.csr_matrix((C.data * (d[C.row] * d[C.col]), (C.row, C.col)), shape=A.shape)
    return As, d


def factor(A, plan, eps, scheme=SECOND_ORDER, stop_after=None, prescaled=False):
    """Approximate factorization of the SPD matrix A (scipy sparse) on `plan`.

    prescaled: factor D A D (module docstring) and apply D M~ D.
    stop_after=l returns (F, B, sizes) right after step l's sparsification:
    the block dict B[(i, j)] of step l's clusters and their current sizes
    (used to compare intermediate blocks)."""
    if scheme not in (FIRST_ORDER, SECOND_ORDER, SUPERFINE):
        raise ValueError(scheme)
    A = sp.csr_matrix(A)
    dscale = None
    if prescaled:
        A, dscale = prescale(A)
    D = plan.depth
    F = Factor(plan.n, scheme, float(eps))
    F.dscale = dscale
    st = plan.steps[D]
    pos = [np.asarray(v, dtype=np.int64) for v in st.verts]
    B = _assemble_leaf_blocks(A, st)
    for l in range(D, -1, -1):
        st = plan.steps[l]
        nI, nc = st.n_interior, st.n_clusters
        fl = 0.0
        shapes = []
        # (a) eliminate interiors
        for s in range(nI):
            nb = [int(w) for w in st.adj[s] if w != s]
            L = _chol(B[(s, s)], l, s, "interior block")
            G = {w: _lsolve(L, B[(s, w)]) for w in nb}
            for i1, w1 in enumerate(nb):
                for w2 in nb[i1:]:
                    C = G[w1].T @ G[w2]
                    B[(w1, w2)] = B[(w1, w2)] - C
                    if w2 != w1:
                        B[(w2, w1)] = B[(w2, w1)] - C.T
            ns = pos[s].size
            ks = int(sum(pos[w].size for w in nb))
            F.ops.append(("interior", pos[s].copy(), L,
                          [(pos[w].copy(), G[w]) for w in nb]))
            F.nnz_L += ns * (ns + 1) // 2 + ns * ks
            fl += ns ** 3 / 3 + ns * ns * ks + ns * ks * ks
            shapes.append((s, ns, ks))
        for key in [k for k in B if k[0] < nI or k[1] < nI]:
            del B[key]
        F.shapes[l] = shapes
        if l == 0:
            F.root_size = int(pos[0].size) if nc else 0
            F.flops[l] = fl
            break
        ranks = []
        if st.sparsified:
            # (b) scale every interface by the Cholesky factor of its diagonal block
            Z = {}
            for p in range(nI, nc):
                Z[p] = _chol(B[(p, p)], l, p, "interface block")
                F.ops.append(("scale", pos[p].copy(), Z[p]))
                a = pos[p].size
                F.nnz_L += a * (a + 1) // 2
                fl += a ** 3 / 3
            for p in range(nI, nc):
                for q in st.adj[p]:
                    q = int(q)
                    if q <= p:
                        continue
                    X = _lsolve(Z[p], B[(p, q)])
                    X = _lsolve(Z[q], X.T).T
                    B[(p, q)] = X
                    B[(q, p)] = X.T.copy()
                B[(p, p)] = np.eye(pos[p].size)
            # (c) sparsify interfaces in (colour, canonical) order
            for p in st.order:
                nb = [int(w) for w in st.adj[p] if w != p and w >= nI]
                a = pos[p].size
                widths = [pos[w].size for w in nb]
                k = int(sum(widths))
                W = np.hstack([B[(p, w)] for w in nb]) if nb else np.zeros((a, 0))
                W = W.reshape(a, k)
                res = cpqr(W, eps, eps * eps if scheme == SUPERFINE else None)
                r, r2 = res["r"], res["r2"]
                Y = res["Y"]
                nbr_pos = np.concatenate([pos[w] for w in nb]) if nb else np.zeros(0, np.int64)
                if scheme == SECOND_ORDER:
                    E = Y[r:, :].copy()
                    fsl = (r, a)
                elif scheme == SUPERFINE:
                    E = Y[r:r2, :].copy()
                    fsl = (r, r2)
                else:
                    E = None
                    fsl = (r, r)
                F.ops.append(("sparsify", pos[p].copy(), res["V"], res["tau"], fsl,
                              nbr_pos, E))
                off = 0
                for w, wd in zip(nb, widths):
                    blk = Y[:r, off:off + wd].copy()
                    B[(p, w)] = blk
                    B[(w, p)] = blk.T.copy()
                    off += wd
                B[(p, p)] = np.eye(r)
                nref = len(res["V"])
                F.nnz_L += a * nref - nref * (nref - 1) // 2 + nref
                if scheme == SECOND_ORDER:
                    F.nnz_L += (a - r) * (k - r)
                elif scheme == SUPERFINE:
                    m2 = r2 - r
                    F.nnz_L += m2 * (k - r) - m2 * (m2 - 1) // 2
                fl += a * a * k + sum(4.0 * (a - j) * (k - j) for j in range(nref))
                ranks.append((p, a, k, r, r2))
                pos[p] = pos[p][:r].copy()
        F.ranks[l] = ranks
        F.flops[l] = fl
        if stop_after == l:
            return F, B, [p_.size for p_ in pos]
        # (d) merge into the clusters of step l-1
        nxt = plan.steps[l - 1]
        new_pos = [np.concatenate([pos[ch] for ch in chs]) if chs else np.zeros(0, np.int64)
                   for chs in nxt.children]
        newB = {}
        for i in range(nxt.n_clusters):
            for j in nxt.adj[i]:
                j = int(j)
                rows = []
                for ci in nxt.children[i]:
                    row = []
                    for cj in nxt.children[j]:
                        blk = B.get((ci, cj))
                        if blk is None:
                            blk = np.zeros((pos[ci].size, pos[cj].size))
                        row.append(blk)
                    rows.append(row)
                newB[(i, j)] = (np.block(rows) if rows and rows[0] else
                                np.zeros((new_pos[i].size, new_pos[j].size)))
                newB[(i, j)] = newB[(i, j)].reshape(new_pos[i].size, new_pos[j].size)
        pos, B = new_pos, newB
    return F


def apply_forward(F, b):
    """z = L^{-1} b (steps depth ... 0, operations in recorded order)."""
    z = np.array(b, dtype=np.float64, copy=True)
    for op in F.ops:
        kind = op[0]
        if kind == "interior":
            _, ps, L, nbrs = op
            zs = _lsolve(L, z[ps])
            z[ps] = zs
            for pw, G in nbrs:
                z[pw] -= G.T @ zs
        elif kind == "scale":
            _, pp, Z = op
            z[pp] = _lsolve(Z, z[pp])
        else:
            _, pp, V, taus, (f0, f1), nbr_pos, E = op
            zp = apply_qt(V, taus, z[pp])
            z[pp] = zp
            if E is not None and f1 > f0:
                z[nbr_pos] -= E.T @ zp[f0:f1]
    return z


def apply_backward(F, z):
    """y = L^{-T} z (the forward operations reversed and transposed)."""
    y = np.array(z, dtype=np.float64, copy=True)
    for op in reversed(F.ops):
        kind = op[0]
        if kind == "interior":
            _, ps, L, nbrs = op
            t = y[ps]
            for pw, G in nbrs:
                t = t - G @ y[pw]
            y[ps] = _ltsolve(L, t)
        elif kind == "scale":
            _, pp, Z = op
            y[pp] = _ltsolve(Z, y[pp])
        else:
            _, pp, V, taus, (f0, f1), nbr_pos, E = op
            yp = y[pp]
            if E is not None and f1 > f0:
                yp[f0:f1] -= E @ y[nbr_pos]
            y[pp] = apply_q(V, taus, yp)
    return y


def apply(F, b):
    """y = M b with M = L^{-T} L^{-1} (prescaled: D L^{-T} L^{-1} D)."""
    if F.dscale is None:
        return apply_backward(F, apply_forward(F, b))
    d = F.dscale if np.ndim(b) == 1 else F.dscale[:, None]
    return d * apply_backward(F, apply_forward(F, d * np.asarray(b, dtype=np.float64)))


def dense_Linv(F):
    """L^{-1} as a dense matrix (tiny problems only)."""
    return apply_forward(F, np.eye(F.n))


def mu(F, A):
    """Memory metric nnz(L) / nnz(A) (Sec. 4 notation)."""
    return F.nnz_L / sp.csr_matrix(A).nnz


def all_ranks(F):
    """Flat list of (step, cluster, a, k, r, r2) in factorization order."""
    out = []
    for l in sorted(F.ranks, reverse=True):
        for rec in F.ranks[l]:
            out.append((l,) + tuple(int(x) for x in rec))
    return out
