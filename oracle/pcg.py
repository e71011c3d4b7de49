"""Preconditioned conjugate gradients as used in the experiments (Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Zero initial guess; convergence is declared when the recursively updated
residual satisfies ||r_k||_2 < tol ||b||_2 (the paper: "falls below" 1e-10).
n_cg is the k at which that happens.  Each column of a multi-column right-hand
side is an independent run.  Hestenes-Stiefel form:

  x = 0, r = b, z = M r, p = z, rho = r.z
  repeat: q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q,
          stop if ||r|| < tol ||b||, z = M r, rho' = r.z, p = z + (rho'/rho) p.
"""
from __future__ import annotations

import numpy as np


class NoConvergence(Exception):
    pass


def pcg(matvec, precond, b, tol=1e-10, maxit=1000, raise_on_fail=False):
    """Solve A x = b for one column b.  Returns (x, iters, history) where
    history[k] = ||r_k|| / ||b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return x, 0, [0.0]
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rho = float(r @ z)
    hist = [1.0]
    for k in range(1, maxit + 1):
        q = matvec(p)
        alpha = rho / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rel = float(np.linalg.norm(r)) / nb
        hist.append(rel)
        if rel < tol:
            return x, k, hist
        z = precond(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    if raise_on_fail:
        raise NoConvergence(f"no convergence in {maxit} iterations (rel {hist[-1]:.3e})")
    return x, maxit, hist


def pcg_multi(matvec, precond, B, tol=1e-10, maxit=1000):
    """Independent PCG runs on the columns of B (n x nrhs)."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    X = np.zeros_like(B)
    iters, hists = [], []
    for j in range(B.shape[1]):
        x, k, h = pcg(matvec, precond, B[:, j], tol, maxit)
        X[:, j] = x
        iters.append(k)
        hists.append(h)
    return X, iters, hists
