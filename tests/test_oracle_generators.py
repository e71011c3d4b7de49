"""Pins of the input generators against closed forms (Sec. 4.1, 4.1.1)."""
import numpy as np
import pytest
import scipy.sparse as sp

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d, high_contrast_2d, rhs


@pytest.mark.parametrize("d", [5, 16, 33])
def test_lap2d_eigenpairs(d):
    # Sec. 4.1.1: x(i,j) = sin(p i pi/(d+1)) sin(p j pi/(d+1)), lambda_p = 8 sin^2(p pi/(2(d+1)))
    p = laplacian_2d(d)
    A = p.scipy()
    i = p.coords[:, 0] + 1
    j = p.coords[:, 1] + 1
    for mode in [1, 2, d // 2 + 1, d]:
        v = np.sin(mode * i * np.pi / (d + 1)) * np.sin(mode * j * np.pi / (d + 1))
        lam = 8 * np.sin(mode * np.pi / (2 * (d + 1))) ** 2
        assert np.allclose(A @ v, lam * v, atol=1e-12 * np.abs(v).max())


def test_lap3d_eigenpair_and_nnz():
    s = 9
    p = laplacian_3d(s)
    A = p.scipy()
    x, y, z = (p.coords[:, a] + 1 for a in range(3))
    for mode in [1, 4, 9]:
        v = np.sin(mode * x * np.pi / (s + 1)) * np.sin(mode * y * np.pi / (s + 1)) * \
            np.sin(mode * z * np.pi / (s + 1))
        lam = 12 * np.sin(mode * np.pi / (2 * (s + 1))) ** 2
        assert np.allclose(A @ v, lam * v, atol=1e-12)
    assert p.nnz == s ** 3 + 6 * s * s * (s - 1)


def test_nnz_closed_forms_of_the_workloads():
    assert laplacian_2d(64).nnz == 20224            # 64^2 + 4*64*63
    p = laplacian_3d(64)
    assert (p.n, p.nnz) == (262144, 1810432)     # 64^3 + 6*64^2*63


def test_vertex_numbering():
    p = laplacian_3d(4, shape=(3, 4, 5))
    vid = p.coords[:, 0] + 3 * (p.coords[:, 1] + 4 * p.coords[:, 2])
    assert np.array_equal(vid, np.arange(p.n))


def test_symmetry_and_sorted_csr():
    for p in [laplacian_2d(7), laplacian_3d(5), fv_diffusion_3d(5, 3.0, 1),
              laplacian_3d(5, (1.0, 1e-2, 1e2)), high_contrast_2d(12, 100.0, 3)]:
        A = p.scipy()
        assert abs(A - A.T).max() == 0.0
        for r in range(p.n):
            c = p.colind[p.rowptr[r]:p.rowptr[r + 1]]
            assert np.all(np.diff(c) > 0)
        assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_fv_constant_coefficient_row_sums():
    # harmonic mean of equal k is k; Dirichlet faces 2k: interior row sums 0,
    # boundary row sums 2k per boundary face
    p = fv_diffusion_3d(6, umax=0.0, seed=5)
    A = p.scipy()
    rs = np.asarray(A.sum(axis=1)).ravel()
    nb = sum((p.coords[:, a] == 0) + (p.coords[:, a] == 5) for a in range(3))
    assert np.allclose(rs, 2.0 * nb)
    off = (A - sp.diags(A.diagonal())).tocsr()
    off.eliminate_zeros()
    assert np.allclose(off.data, -1.0)


def test_fv_harmonic_faces():
    p = fv_diffusion_3d(4, umax=3.0, seed=7)
    u = np.random.default_rng(7).uniform(-3, 3, size=(4, 4, 4)).ravel()
    k = 10.0 ** u
    A = p.scipy()
    assert np.isclose(-A[0, 1], 2 * k[0] * k[1] / (k[0] + k[1]), rtol=1e-14)
    assert np.isclose(-A[0, 16], 2 * k[0] * k[16] / (k[0] + k[16]), rtol=1e-14)


def test_rhs_seeded():
    a = rhs(100, 3, 2001)
    b = rhs(100, 3, 2001)
    assert a.flags.f_contiguous and np.array_equal(a, b)
    assert not np.array_equal(a, rhs(100, 3, 2002))
