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


def _crown(m):
    """K_{m,m} minus a perfect matching, vertices u_i = 2i, v_i = 2i + 1: greedy
    colouring in index order needs m colours, the graph is bipartite."""
    adj = {x: [] for x in range(2 * m)}
    for i in range(m):
        for j in range(m):
            if i != j:
                adj[2 * i].append(2 * j + 1)
                adj[2 * j + 1].append(2 * i)
    return adj


def test_dsatur_on_graphs_with_known_chromatic_numbers():
    # DSATUR is exact on bipartite graphs (the crown defeats plain greedy)
    adj = _crown(6)
    col = nd.dsatur_colour(adj, list(adj), {x: 1 for x in adj})
    assert max(col.values()) + 1 == 2
    # odd cycle: 3 colours; complete graph K_5: 5
    cyc = {x: [(x - 1) % 7, (x + 1) % 7] for x in range(7)}
    assert max(nd.dsatur_colour(cyc, list(cyc), {x: 1 for x in cyc}).values()) + 1 == 3
    k5 = {x: [y for y in range(5) if y != x] for x in range(5)}
    assert sorted(nd.dsatur_colour(k5, list(k5), {x: 1 for x in k5}).values()) == [0, 1, 2, 3, 4]


def test_dsatur_tie_breaks():
    # first pick: largest weight, then lowest index; it takes colour 0 and its
    # neighbours then lead by saturation
    path = {0: [1], 1: [0, 2], 2: [1, 3], 3: [2]}
    col = nd.dsatur_colour(path, [0, 1, 2, 3], {0: 1, 1: 1, 2: 5, 3: 1})
    assert col[2] == 0 and col[1] == 1 and col[3] == 1 and col[0] == 0
    col = nd.dsatur_colour(path, [0, 1, 2, 3], {0: 1, 1: 1, 2: 1, 3: 1})
    assert col[0] == 0 and col[1] == 1 and col[2] == 0 and col[3] == 1


def test_plan_colouring_is_proper_and_ordered():
    p = laplacian_3d(12)
    plan = nd.analyze(p.rowptr, p.colind, p.coords, 6)
    for st in plan.steps.values():
        nI = st.n_interior
        for p_ in range(nI, st.n_clusters):
            assert all(st.colour[q] != st.colour[p_] for q in st.adj[p_] if q >= nI and q != p_)
        used = sorted({int(c) for c in st.colour[nI:]})
        assert used == list(range(len(used)))
        assert st.order == sorted(range(nI, st.n_clusters), key=lambda x: (st.colour[x], x))


# --- coordinate-free reading: landmark hop distances -------------------------

@pytest.mark.parametrize("W,H", [(7, 5), (8, 8), (13, 4), (1, 9)])
def test_graph_coords_closed_form_2d(W, H):
    # On a W x H five-point grid (vertex id = y W + x) hop distance is the
    # Manhattan distance: l0 is the far corner (W-1, H-1), l1 the corner
    # (0, 0), and l2 the lowest-id vertex on the anti-diagonal x + y =
    # floor((W + H - 2) / 2), i.e. the one with the smallest y.
    p = laplacian_2d(W, H)
    xy = nd.graph_coords(p.rowptr, p.colind)
    x, y = p.coords[:, 0], p.coords[:, 1]
    s = (W + H - 2) // 2
    ys = max(0, s - (W - 1))
    xs = s - ys
    assert np.array_equal(xy[:, 0], (W - 1 - x) + (H - 1 - y))
    assert np.array_equal(xy[:, 1], x + y)
    assert np.array_equal(xy[:, 2], np.abs(x - xs) + np.abs(y - ys))


def test_graph_coords_closed_form_3d():
    m = 6
    p = laplacian_3d(m)
    xyz = nd.graph_coords(p.rowptr, p.colind)
    x, y, z = p.coords[:, 0], p.coords[:, 1], p.coords[:, 2]
    s = 3 * (m - 1) // 2               # lowest id on x + y + z = s: z = 0, then y small
    zs = 0
    ys = max(0, s - (m - 1))
    xs = s - ys
    assert np.array_equal(xyz[:, 0], 3 * (m - 1) - (x + y + z))
    assert np.array_equal(xyz[:, 1], x + y + z)
    assert np.array_equal(xyz[:, 2], np.abs(x - xs) + np.abs(y - ys) + np.abs(z - zs))


def test_graph_coords_unreachable_and_plan():
    # two disjoint grids: vertices of the other component sit at distance n
    a, b = laplacian_2d(6, 4), laplacian_2d(5, 5)
    n = a.n + b.n
    rowptr = np.concatenate([a.rowptr, a.rowptr[-1] + b.rowptr[1:]])
    colind = np.concatenate([a.colind, b.colind + a.n])
    xy = nd.graph_coords(rowptr, colind)
    # l0: farthest from vertex 0 is unreachable, lowest id = first vertex of b
    assert np.all(xy[:a.n, 0] == n) and xy[a.n, 0] == 0
    plan = nd.analyze(rowptr, colind, None, 3, 1)
    nd.check_plan(plan, rowptr, colind)
    assert np.array_equal(plan.perm[np.argsort(plan.perm)], np.arange(n))
