"""Pins of the oracle's early-stopping column-pivoted QR (Alg. 1, Sec. 3.1)
against LAPACK's pivoted QR (through scipy) and the algebra of reflectors."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.dense import cpqr, householder, apply_q, apply_qt


@pytest.mark.parametrize("a,k,seed", [(7, 20, 0), (20, 7, 1), (16, 16, 2), (40, 130, 3), (1, 5, 4)])
def test_full_cpqr_matches_lapack(a, k, seed):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((a, k)) * np.exp(-0.3 * np.arange(k))[None, :]
    res = cpqr(W, 0.0)
    _, R, piv = sla.qr(W, pivoting=True)
    m = min(a, k)
    assert res["r"] == m
    assert res["piv"] == list(piv[:m])
    assert np.allclose(res["diag"], np.abs(np.diag(R))[:m], rtol=1e-12)


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3])
def test_early_stop_is_truncation(eps):
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((90, 30)))
    W = U @ np.diag(10.0 ** -np.linspace(0, 5, 30)) @ V.T
    res = cpqr(W, eps)
    _, R, piv = sla.qr(W, pivoting=True)
    d = np.abs(np.diag(R))
    r_ref = int(np.argmax(d < eps * d[0])) if (d < eps * d[0]).any() else d.size
    assert res["r"] == r_ref
    assert res["piv"] == list(piv[:r_ref])
    # the dropped part is below the threshold: max trailing column norm < eps |R00|
    E = res["Y"][res["r"]:]
    assert np.linalg.norm(E, axis=0).max() < eps * d[0]


def test_reflectors_reconstruct_W():
    rng = np.random.default_rng(9)
    W = rng.standard_normal((12, 40))
    res = cpqr(W, 1e-1)
    Q = apply_q(res["V"], res["tau"], np.eye(12))
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-14)
    assert np.allclose(Q @ res["Y"], W, atol=1e-13)
    assert np.allclose(apply_qt(res["V"], res["tau"], W), res["Y"], atol=1e-13)
    # pivot columns are exactly beta e_j: zero below row j, and zero in E
    Y = res["Y"]
    for j, c in enumerate(res["piv"]):
        assert (Y[j + 1:, c] == 0).all() and abs(Y[j, c]) == res["diag"][j]


def test_householder_convention():
    x = np.array([3.0, 4.0])
    v, tau, beta = householder(x)
    assert beta == -5.0 and v[0] == 1.0
    Hx = x - tau * v * (v @ x)
    assert np.allclose(Hx, [beta, 0.0])
    v, tau, beta = householder(np.array([-3.0, 4.0]))
    assert beta == 5.0
    v, tau, beta = householder(np.array([0.0, 2.0]))   # sign(0) = +1
    assert beta == -2.0
    v, tau, beta = householder(np.zeros(3))
    assert tau == 0.0 and beta == 0.0


def test_ties_go_to_lowest_index():
    # columns 1 and 3 are the same vector: equal norms, pivot = 1
    rng = np.random.default_rng(0)
    c = rng.standard_normal(5)
    W = np.stack([0.5 * c, c, 0.1 * rng.standard_normal(5), c], axis=1)
    assert cpqr(W, 0.0)["piv"][0] == 1
    # a mirrored column with a norm equal up to rounding is still a tie
    W2 = np.stack([c[::-1] * (1 + 1e-15), c], axis=1)
    assert cpqr(W2, 0.0)["piv"][0] == 0


def test_degenerate():
    assert cpqr(np.zeros((4, 0)), 0.1)["r"] == 0
    assert cpqr(np.zeros((0, 4)), 0.1)["r"] == 0
    assert cpqr(np.zeros((3, 5)), 0.0)["r"] == 0        # a zero pivot always stops
    W = np.outer(np.arange(1.0, 5.0), np.ones(6))      # rank one
    res = cpqr(W, 0.0)
    assert res["r"] >= 1 and res["diag"][0] == pytest.approx(np.sqrt(30.0))


def test_superfine_extends_the_same_run():
    rng = np.random.default_rng(3)
    W = rng.standard_normal((25, 60)) * (10.0 ** -np.linspace(0, 6, 60))[None, :]
    r1 = cpqr(W, 1e-2)
    r2 = cpqr(W, 1e-2, 1e-4)
    assert r2["r"] == r1["r"] and r2["r2"] >= r2["r"]
    assert r2["piv"][:r1["r"]] == r1["piv"]
    assert np.array_equal(r2["Y"][:r1["r"]], r1["Y"][:r1["r"]])
    d = np.array(r2["diag"])
    assert (d[r2["r"]:] < 1e-2 * d[0]).all() and (d >= 1e-4 * d[0]).all()
