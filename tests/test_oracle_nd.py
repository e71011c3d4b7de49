"""Pins of the oracle's nested dissection and cluster structure.

The paper's partitioner is algebraic and defined elsewhere, so parity with it
is unpinned; these tests check the structural properties the method needs
(Sec. 3, Fig. 1): separators separate, interiors of a step never interact,
every vertex sits in one cluster, every interface maps to one parent, and
interfaces of one colour are never adjacent.
"""
import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d
from oracle import nd


@pytest.mark.parametrize("make,depth", [
    (lambda: laplacian_2d(64), 6),
    (lambda: laplacian_2d(17, 9), 5),
    (lambda: laplacian_3d(12), 6),
    (lambda: laplacian_3d(5, shape=(7, 3, 9)), 8),
    (lambda: fv_diffusion_3d(8, 3.0, 1), 5),
])
def test_structure(make, depth):
    p = make()
    plan = nd.analyze(p.rowptr, p.colind, p.coords, depth)
    nd.check_plan(plan, p.rowptr, p.colind)
    # every vertex alive at step l is in exactly one step-l cluster: the sizes add up
    sizes = {depth: np.array([v.size for v in plan.steps[depth].verts])}
    for l in range(depth - 1, -1, -1):
        st = plan.steps[l]
        prev = sizes[l + 1]
        sizes[l] = np.array([prev[ch].sum() if ch else 0 for ch in st.children])
        assert sizes[l].sum() == (plan.lvl <= l).sum()


def test_root_cut_on_64x64():
    # x extent and y extent tie at 63 -> axis 0; sorted x of index 2048 is 32:
    # L = {x < 32}, separator = the column x = 31
    p = laplacian_2d(64)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 6)
    root = plan.nodes[0]
    assert (root.ax, root.t, root.le) == (0, 32.0, False)
    assert np.array_equal(np.sort(root.sep), np.flatnonzero(p.coords[:, 0] == 31))
    assert (plan.lvl[p.coords[:, 0] == 31] == 0).all()
    # the next cuts split y
    assert plan.nodes[root.left].ax == 1 and plan.nodes[root.right].ax == 1


def test_leaf_sizes_and_levels():
    p = laplacian_3d(16)
    D = 6
    plan = nd.analyze(p.rowptr, p.colind, p.coords, D)
    st = plan.steps[D]
    assert st.n_interior == 2 ** D
    cells = p.n / 2 ** D
    leaf = np.array([v.size for v in st.verts[:st.n_interior]])
    assert leaf.max() <= cells and leaf.min() > 0
    assert set(np.unique(plan.lvl)) == set(range(D + 1))


def test_deterministic():
    p = laplacian_3d(10)
    a = nd.analyze(p.rowptr, p.colind, p.coords, 7)
    b = nd.analyze(p.rowptr, p.colind, p.coords, 7)
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.path, b.path)
    for l in a.steps:
        assert a.steps[l].keys == b.steps[l].keys
        assert np.array_equal(a.steps[l].colour, b.steps[l].colour)


def test_degenerate_inputs():
    # a single vertex, a line of equal coordinates (extent 0), depth 0
    from synthetic.problems import Problem
    p = laplacian_2d(1)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 4)
    assert plan.steps[4].n_clusters == 1
    q = laplacian_2d(5)
    coords = np.zeros_like(q.coords)
    plan = nd.analyze(q.rowptr, q.colind, coords, 3)
    assert len(plan.nodes) == 1 and (plan.lvl == 3).all()
    plan = nd.analyze(q.rowptr, q.colind, q.coords, 0)
    assert plan.steps[0].n_clusters == 1 and plan.steps[0].n_interior == 1
    del Problem


def test_colouring_is_greedy_smallest_free():
    p = laplacian_3d(12)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 6)
    for st in plan.steps.values():
        nI = st.n_interior
        for p_ in range(nI, st.n_clusters):
            earlier = {int(st.colour[q]) for q in st.adj[p_] if nI <= q < p_}
            c = 0
            while c in earlier:
                c += 1
            assert st.colour[p_] == c
        assert st.order == sorted(range(nI, st.n_clusters), key=lambda x: (st.colour[x], x))
