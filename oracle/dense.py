"""Early-stopping column-pivoted Householder QR (Alg. 1, Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given the a x k coupling W = A_pw of an interface, QR with column pivoting
(Businger-Golub) gives W P = Q R.  The run stops at the first pivot whose
|R(j,j)| falls below eps |R(0,0)| (first-order and full second-order), or
below eps^2 |R(0,0)| (superfine second order, which also reports where the
eps test first failed).  Readings (the paper is silent on these):

* The trailing column norms are recomputed exactly at every step (no
  downdating).
* Pivot: the trailing column of largest norm; columns whose squared norm is
  within a relative TIE_RTOL of the largest count as tied, and the tie goes to
  the lowest original column index.  This keeps the pivot sequence insensitive
  to summation-order rounding, which otherwise breaks exact symmetric ties of
  grid problems differently on different machines.
* Householder reflector H = I - tau v v^T with v[0] = 1 and
  H x = beta e_1, beta = -sign(x_0) ||x||, sign(0) = +1; a zero column gives
  tau = 0 (H = I).
* Rank r = number of leading pivots with |R(j,j)| > 0 and
  |R(j,j)| >= eps |R(0,0)| (a pivot equal to 0 always stops the run; so an
  empty or all-zero W has rank 0, and eps = 0 keeps every nonzero pivot).

The reflectors are applied to the columns of W in place, without permuting
them, so the result Y = Q^T W is in the original column order:
Y[:r] = Q_c^T W = [R_cc R_cf] P^T, and Y[r:] = Q_f^T W = [0 R_ff] P^T = E.
The pivot columns are stored exactly as beta e_j.
"""
from __future__ import annotations

import numpy as np

TIE_RTOL = 1e-8


def householder(x):
    """(v, tau, beta) with (I - tau v v^T) x = beta e_1 and v[0] = 1."""
    nrm = float(np.sqrt(np.dot(x, x)))
    v = np.zeros_like(x)
    if x.size:
        v[0] = 1.0
    if nrm == 0.0:
        return v, 0.0, 0.0
    alpha = float(x[0])
    beta = -nrm if alpha >= 0.0 else nrm
    v[1:] = x[1:] / (alpha - beta)
    tau = (beta - alpha) / beta
    return v, tau, beta


def cpqr(W, eps, eps2=None):
    """Early-stopping CPQR of W (a x k).

    Returns a dict with
      Y     : Q^T W (a x k, original column order) after all reflectors,
      V, tau: the reflectors (V[j] has length a - j, V[j][0] = 1),
      piv   : pivot columns (original indices) in order,
      r     : rank at tolerance eps,
      r2    : rank at tolerance eps2 (== r when eps2 is None),
      diag  : |R(j,j)| of every reflector applied.
    """
    W = np.asarray(W, dtype=np.float64)
    a, k = W.shape
    Y = W.copy()
    remaining = np.arange(k)
    V, taus, piv, diag = [], [], [], []
    stop_tol = eps if eps2 is None else eps2
    r = None
    R00 = 0.0
    for j in range(min(a, k)):
        nrm2 = np.einsum("ij,ij->j", Y[j:, remaining], Y[j:, remaining])
        m = nrm2.max()
        cand = remaining[nrm2 >= m * (1.0 - TIE_RTOL)].min()
        x = Y[j:, cand].copy()
        nrm = float(np.sqrt(np.dot(x, x)))
        if j == 0:
            R00 = nrm
        if nrm == 0.0 or nrm < stop_tol * R00:
            break
        if r is None and nrm < eps * R00:
            r = j
        v, tau, beta = householder(x)
        rest = remaining[remaining != cand]
        if rest.size:
            blk = Y[j:, rest]
            Y[j:, rest] = blk - tau * np.outer(v, v @ blk)
        Y[j, cand] = beta
        Y[j + 1:, cand] = 0.0
        V.append(v)
        taus.append(tau)
        piv.append(int(cand))
        diag.append(abs(beta))
        remaining = rest
    nref = len(V)
    if r is None:
        r = nref
    return dict(Y=Y, V=V, tau=taus, piv=piv, r=r, r2=nref, diag=diag)


def apply_qt(V, taus, x):
    """x <- Q^T x for Q = H_0 H_1 ... H_{m-1} (x: vector or matrix, rows)."""
    x = x.copy()
    for j, (v, tau) in enumerate(zip(V, taus)):
        if tau != 0.0:
            x[j:] -= tau * np.outer(v, v @ x[j:]) if x.ndim == 2 else tau * v * (v @ x[j:])
    return x


def apply_q(V, taus, x):
    """x <- Q x."""
    x = x.copy()
    for j in range(len(V) - 1, -1, -1):
        v, tau = V[j], taus[j]
        if tau != 0.0:
            x[j:] -= tau * np.outer(v, v @ x[j:]) if x.ndim == 2 else tau * v * (v @ x[j:])
    return x
