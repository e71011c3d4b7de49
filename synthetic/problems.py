"""Seeded generators for the model problems of the paper's experiments (Sec. 4.1)
and for the synthetic workloads this project measures.

Every matrix is symmetric positive definite, stored as CSR with both triangles
and the diagonal (int64 row pointers, int32 column indices, float64 values,
column indices sorted within each row).  Vertex ``(x, y[, z])`` of an
``sx x sy [x sz]`` grid has id ``x + sx*(y + sy*z)`` and unit-spaced
coordinates ``(x, y[, z])``.

Discretizations:

* ``laplacian_2d``: the 5-point Dirichlet Laplacian with diagonal 4 and
  off-diagonals -1, unscaled.  Its eigenvectors are products of sines with
  eigenvalues ``8 sin^2(p pi / (2(d+1)))`` on the (p, p) modes (Sec. 4.1.1).
* ``laplacian_3d``: the 7-point analogue (diagonal ``2*sum(w)``, off-diagonal
  ``-w_axis``); axis weights make the anisotropic variant.
* ``fv_diffusion_3d`` / ``high_contrast_2d``: cell-centred finite volumes with
  harmonic-mean face transmissibility ``2 k_a k_b / (k_a + k_b)`` and Dirichlet
  boundary faces ``2 k_c`` (unit spacing).

Nothing here performs any step of the factorization; the module only builds
inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.ndimage import gaussian_filter


@dataclass
class Problem:
    name: str
    shape: tuple          # grid sizes, x first
    rowptr: np.ndarray    # int64 [n+1]
    colind: np.ndarray    # int32 [nnz]
    vals: np.ndarray      # float64 [nnz]
    coords: np.ndarray    # float64 [n, dim], C-contiguous
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    @property
    def dim(self) -> int:
        return int(self.coords.shape[1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))


def _coords(shape):
    # numpy arrays are indexed [z, y, x] so that C-order flattening gives
    # id = x + sx*(y + sy*z)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape[::-1]], indexing="ij")
    cols = [g.ravel() for g in grids[::-1]]  # x first
    return np.ascontiguousarray(np.stack(cols, axis=1))


def _assemble(shape, face_t, bnd_t):
    """face_t[a]: transmissibility of the faces normal to axis a (x=0), array in
    [z, y, x] index order with size s_a - 1 along that axis.  bnd_t[a]: the
    diagonal contribution of a missing neighbour across a boundary face normal
    to axis a, array over cells."""
    dim = len(shape)
    n = int(np.prod(shape))
    ids = np.arange(n, dtype=np.int64).reshape(shape[::-1])
    diag = np.zeros(shape[::-1], dtype=np.float64)
    rows, cols, vals = [], [], []
    for a in range(dim):
        ax = dim - 1 - a  # numpy axis of grid axis a
        t = face_t[a]
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, shape[a] - 1)
        hi[ax] = slice(1, shape[a])
        i0 = ids[tuple(lo)].ravel()
        i1 = ids[tuple(hi)].ravel()
        tv = t.ravel()
        rows += [i0, i1]
        cols += [i1, i0]
        vals += [-tv, -tv]
        diag[tuple(lo)] += t
        diag[tuple(hi)] += t
        # boundary faces at both ends of the axis
        first = [slice(None)] * dim
        last = [slice(None)] * dim
        first[ax] = slice(0, 1)
        last[ax] = slice(shape[a] - 1, shape[a])
        diag[tuple(first)] += bnd_t[a][tuple(first)]
        diag[tuple(last)] += bnd_t[a][tuple(last)]
    rows.append(ids.ravel())
    cols.append(ids.ravel())
    vals.append(diag.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    m = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (np.ascontiguousarray(m.indptr.astype(np.int64)),
            np.ascontiguousarray(m.indices.astype(np.int32)),
            np.ascontiguousarray(m.data.astype(np.float64)))


def _stencil(shape, weights):
    dim = len(shape)
    face_t, bnd_t = [], []
    for a in range(dim):
        fs = list(shape[::-1])
        fs[dim - 1 - a] -= 1
        face_t.append(np.full(fs, float(weights[a])))
        bnd_t.append(np.full(shape[::-1], float(weights[a])))
    return face_t, bnd_t


def laplacian_2d(d: int, sy: int | None = None) -> Problem:
    """5-point Dirichlet Laplacian on a d x sy grid (diag 4, off -1)."""
    shape = (d, d if sy is None else sy)
    ft, bt = _stencil(shape, (1.0, 1.0))
    rp, ci, v = _assemble(shape, ft, bt)
    return Problem(f"lap2d_{shape[0]}x{shape[1]}", shape, rp, ci, v, _coords(shape))


def laplacian_3d(s: int, weights=(1.0, 1.0, 1.0), shape=None) -> Problem:
    """7-point Laplacian on an s^3 grid, axis weights (wx, wy, wz):
    off-diagonal -w_axis, diagonal 2*(wx+wy+wz) (Dirichlet)."""
    shape = (s, s, s) if shape is None else tuple(shape)
    ft, bt = _stencil(shape, weights)
    rp, ci, v = _assemble(shape, ft, bt)
    tag = "lap3d" if tuple(weights) == (1.0, 1.0, 1.0) else "aniso3d"
    return Problem(f"{tag}_{shape[0]}x{shape[1]}x{shape[2]}", shape, rp, ci, v,
                   _coords(shape), {"weights": tuple(float(w) for w in weights)})


def _fv(shape, k):
    dim = len(shape)
    face_t, bnd_t = [], []
    for a in range(dim):
        ax = dim - 1 - a
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, shape[a] - 1)
        hi[ax] = slice(1, shape[a])
        ka, kb = k[tuple(lo)], k[tuple(hi)]
        face_t.append(2.0 * ka * kb / (ka + kb))
        bnd_t.append(2.0 * k)
    return _assemble(shape, face_t, bnd_t)


def fv_diffusion_3d(s: int, umax: float = 3.0, seed: int = 1002) -> Problem:
    """Cell-centred 7-point FV diffusion on s^3 cells with k = 10**u,
    u ~ U[-umax, umax] i.i.d. per cell drawn in C order (z, y, x)."""
    shape = (s, s, s)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-umax, umax, size=(s, s, s))
    k = 10.0 ** u
    rp, ci, v = _fv(shape, k)
    return Problem(f"fv3d_{s}_u{umax:g}", shape, rp, ci, v, _coords(shape),
                   {"umax": umax, "seed": seed})


def high_contrast_2d(d: int, rho: float, seed: int = 0, sigma: float = 2.0) -> Problem:
    """The 2D high-contrast field of Sec. 4.1: U(0,1) per cell, Gaussian blur
    (std sigma, reflecting boundary), quantised to rho / 1/rho at 0.5; then
    cell-centred FV with harmonic-mean faces and Dirichlet faces 2 a_c."""
    shape = (d, d)
    rng = np.random.default_rng(seed)
    a_hat = gaussian_filter(rng.uniform(0.0, 1.0, size=(d, d)), sigma=sigma, mode="reflect")
    a = np.where(a_hat >= 0.5, rho, 1.0 / rho)
    rp, ci, v = _fv(shape, a)
    return Problem(f"hc2d_{d}_rho{rho:g}", shape, rp, ci, v, _coords(shape),
                   {"rho": rho, "seed": seed})


def rhs(n: int, nrhs: int = 1, seed: int = 2000) -> np.ndarray:
    """Right-hand sides ~ N(0,1), shape (n, nrhs), Fortran order (column j is
    one right-hand side, contiguous)."""
    b = np.random.default_rng(seed).standard_normal((n, nrhs))
    return np.asfortranarray(b)


# Named workloads: matrix family, size and the solver settings they run with.
WORKLOADS = {
    # 2D 5-point, 64^2, depth 6, eps 1e-2, full second order, FP64, tol 1e-12
    "lap2d_64": dict(make=lambda: laplacian_2d(64), depth=6, skip=4, eps=1e-2,
                     nrhs=1, rhs_seed=2000, tol=1e-12),
    # 3D 7-point, 64^3, depth 12, eps 1e-2, 4 RHS, tol 1e-10
    "lap3d_64": dict(make=lambda: laplacian_3d(64), depth=12, skip=4, eps=1e-2,
                     nrhs=4, rhs_seed=2001, tol=1e-10),
    # 3D FV high contrast, 128^3, k = 10^U[-3,3], depth 15, eps 1e-2, tol 1e-10
    "fv3d_128": dict(make=lambda: fv_diffusion_3d(128, 3.0, 1002), depth=15, skip=4,
                     eps=1e-2, nrhs=1, rhs_seed=2002, tol=1e-10),
}


def batch_problems(count2d: int = 128, count3d: int = 128, seed: int = 3000):
    """Independent problems of the batch workload: count2d 2D 5-point
    Laplacians with side ~ U{32..256} and count3d anisotropic 3D 7-point
    operators with side ~ U{16..48} and axis weights (1, 1e-2, 1e2), sides
    drawn from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    s2 = rng.integers(32, 257, size=count2d)
    s3 = rng.integers(16, 49, size=count3d)
    probs = [laplacian_2d(int(d)) for d in s2]
    probs += [laplacian_3d(int(d), weights=(1.0, 1e-2, 1e2)) for d in s3]
    return probs


def workload(name: str):
    """Return (problem, settings dict) of a named workload."""
    w = dict(WORKLOADS[name])
    prob = w.pop("make")()
    return prob, w


def serve_stream(count: int = 48, rate: float = 50.0, reuse: float = 0.3, side=(32, 96),
                 umax: float = 2.0, nrhs_max: int = 16, seed: int = 4000):
    """Requests of the serving workload, in arrival order: Poisson arrivals at
    `rate` per second; with probability `reuse` a request reuses the matrix of
    a uniformly drawn earlier request (the first one never does), otherwise it
    brings a new 3D FV diffusion matrix with side ~ U{side} and coefficient
    exponents u ~ U[-umax, umax]; nrhs ~ U{1..nrhs_max}.  Each entry is a dict
    with arrival time t (s), key, side, matrix seed, nrhs and rhs seed; the
    matrix of a key is fv_diffusion_3d(side, umax, mseed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out, keys = [], []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        if keys and rng.random() < reuse:
            key = keys[int(rng.integers(len(keys)))]
            s, ms = key
        else:
            s = int(rng.integers(side[0], side[1] + 1))
            ms = seed + 1 + i
            key = (s, ms)
            keys.append(key)
        out.append(dict(t=t, key=key, side=s, mseed=ms, umax=umax,
                        nrhs=int(rng.integers(1, nrhs_max + 1)), rhs_seed=seed + 100000 + i))
    return out


def poisson_modes(d: int):
    """Mode numbers p = floor(1.25^k) <= d, k = 0, 1, ..., without repeats."""
    out, k = [], 0
    while True:
        p = int(np.floor(1.25 ** k))
        if p > d:
            return out
        if not out or p != out[-1]:
            out.append(p)
        k += 1


def poisson_eigvec(d: int, p: int):
    """Unit eigenvector of the d x d 5-point Dirichlet Laplacian for the grid
    function sin(p i pi/(d+1)) sin(p j pi/(d+1)), i, j = 1..d (vertex id
    x + d y with i = x + 1, j = y + 1), and its eigenvalue
    8 sin^2(p pi / (2 (d+1)))."""
    s = np.sin(p * np.arange(1, d + 1) * np.pi / (d + 1))
    v = np.outer(s, s).reshape(-1)     # row y, column x: index x + d y
    v /= np.linalg.norm(v)
    return v, 8.0 * np.sin(p * np.pi / (2.0 * (d + 1))) ** 2


SKETCH_ROWS = 256
_SKETCH_CHUNK = 1 << 16


def sketch(X, seed: int = 77, m: int = SKETCH_ROWS) -> np.ndarray:
    """Seeded Gaussian projection S^T X of the columns of X (n or n x nrhs),
    S ~ N(0,1)^(n x m).  S is drawn in row chunks of 65,536 (chunk c from
    default_rng([seed, c])), so any n is projected in bounded memory and the
    same S is drawn for the same (n, seed, m).  Returns m x nrhs.  For any
    vector v, ||S^T v|| / sqrt(m) estimates ||v|| (to about 10 % at m = 256),
    so ||S^T (x - y)|| / ||S^T y|| estimates the relative error of x against y
    over all n entries.  A test-side projection: no step of the method."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n = X.shape[0]
    out = np.zeros((m, X.shape[1]))
    for c, lo in enumerate(range(0, n, _SKETCH_CHUNK)):
        hi = min(n, lo + _SKETCH_CHUNK)
        S = np.random.default_rng([seed, c]).standard_normal((hi - lo, m))
        out += S.T @ X[lo:hi]
    return out
