"""Geometric nested dissection, clusters per step, block structure and colouring.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's spaND partitioning is algebraic and defined in the base spaND paper
(Sec. 3); this oracle uses the coordinate-bisection reading below instead.  The
GPU library implements the same reading independently and must reproduce its
output bit for bit.  Parity against the paper's own partitioner is unpinned.

Reading (the paper is silent on these points):

* Node N at depth d holding vertex set V is a leaf when d == depth, |V| <= 1,
  or every coordinate extent of V is 0.  Otherwise the cut axis is the axis of
  largest extent (lowest axis on ties); V is sorted by (x_axis, vertex id) and
  t is x_axis of the element at index |V| // 2.  L = {x_axis < t}; if that is
  empty, L = {x_axis <= t} (the "<=" flag).  If R = V \\ L is empty, N is a leaf.
* The separator of N is S_N = {v in L : some off-diagonal entry (v, u) of A
  has u in R}.  The left child holds L \\ S_N (path bit 0), the right child R
  (path bit 1).
* Levels: lvl(v) = depth for leaf vertices, lvl(v) = d for v in S_N.
* Paths are depth-bit integers, the bit of tree depth e at position
  depth-1-e.  A leaf vertex gets its leaf's path, zero padded.  A separator
  vertex of N gets path(N), then bit 0, then the bits of a walk down N's left
  subtree that compares the vertex with each node's stored cut, zero padded
  when the walk reaches a leaf.
* Step l (l = depth ... 0): the remaining vertices are those with lvl <= l.
  Interiors are the vertices with lvl == l grouped by prefix_l(path) =
  path >> (depth - l).  Interfaces are the vertices with lvl < l grouped by
  (lvl, prefix_l).  Canonical order: interiors by prefix, then interfaces by
  (lvl, prefix).
* Variables of a step-depth cluster are its vertices in ascending id.  A
  step-l cluster (l < depth) concatenates the current (coarse) variables of
  its step-(l+1) children in their canonical order.
* Two clusters are adjacent when A couples them, or when both border an
  interior eliminated at this or an earlier step (symbolic fill); adjacency is
  lifted to parents at every merge.  Sparsification keeps the structure.
* Interfaces of a sparsified step are processed by (colour, canonical index),
  with colours from a DSATUR colouring of the interface adjacency graph:
  repeatedly the uncoloured interface with the most distinct colours among its
  coloured neighbours is taken (ties: the one holding more vertices of A, then
  the lower canonical index) and given the smallest colour none of its
  coloured neighbours has.  Interfaces of one colour are never adjacent, so
  their relative order cannot change the result; fewer colours mean fewer
  sequential sparsification rounds.  (Alg. 2 writes a FORALL over interfaces, which reads as
  order independent; it is not, for adjacent interfaces.)
* Sparsified steps (scaling + sparsification, Alg. 2): 1 <= l <= depth - skip;
  the paper skips the first four levels (Sec. 4), so skip defaults to 4.

Coordinate-free analysis (the paper's partition works on the matrix alone,
Sec. 3; reading of this project): when no coordinates are given, each vertex
gets as coordinates its hop distances in the graph of A to three landmarks
chosen by farthest-point sampling -- l0 the vertex farthest from vertex 0, l1
the vertex farthest from l0, l2 the vertex maximising the distance to the
nearer of l0 and l1 (lowest vertex id on ties, unreachable vertices at
distance n) -- and the bisection above runs on those.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Node:
    depth: int
    bits: int                 # path of the node: `depth` bits
    verts: np.ndarray
    leaf: bool = True
    ax: int = -1
    t: float = 0.0
    le: bool = False          # True: left = {x_ax <= t}
    left: int = -1
    right: int = -1
    sep: np.ndarray | None = None


@dataclass
class Step:
    l: int
    keys: list                # (kind, lvl, prefix); kind 0 = interior, 1 = interface
    n_interior: int
    adj: list                 # per cluster: sorted int array of adjacent clusters (incl. self)
    colour: np.ndarray        # per cluster; -1 for interiors
    sparsified: bool
    order: list               # interface cluster ids in sparsification order
    children: list | None     # l < depth: per cluster, step-(l+1) cluster ids in order
    verts: list | None        # l == depth: per cluster, sorted vertex ids

    @property
    def n_clusters(self) -> int:
        return len(self.keys)


@dataclass
class Plan:
    n: int
    depth: int
    skip: int
    lvl: np.ndarray
    path: np.ndarray
    perm: np.ndarray          # elimination permutation (for parity reports)
    nodes: list
    steps: dict = field(default_factory=dict)   # l -> Step


def _rows_touching(rowptr, colind, rows, mask):
    """For each vertex in `rows`, whether any of its neighbours has mask True."""
    if rows.size == 0:
        return np.zeros(0, dtype=bool)
    starts = rowptr[rows]
    lens = rowptr[rows + 1] - starts
    tot = int(lens.sum())
    if tot == 0:
        return np.zeros(rows.size, dtype=bool)
    offs = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
    idx = offs + np.arange(tot)
    hits = mask[colind[idx]].astype(np.int64)
    owner = np.repeat(np.arange(rows.size), lens)
    return np.bincount(owner, weights=hits, minlength=rows.size) > 0


def dissect(rowptr, colind, coords, depth):
    """Build the nested-dissection tree; returns the list of nodes (root first)."""
    n = coords.shape[0]
    nodes = [Node(0, 0, np.arange(n, dtype=np.int64))]
    mask = np.zeros(n, dtype=bool)
    stack = [0]
    while stack:
        ni = stack.pop()
        nd = nodes[ni]
        V = nd.verts
        if nd.depth == depth or V.size <= 1:
            continue
        X = coords[V]
        ext = X.max(axis=0) - X.min(axis=0)
        if ext.max() == 0.0:
            continue
        ax = int(np.argmax(ext))          # first maximum: lowest axis on ties
        xa = X[:, ax]
        order = np.lexsort((V, xa))
        t = xa[order[V.size // 2]]
        le = False
        inL = xa < t
        if not inL.any():
            inL = xa <= t
            le = True
        if inL.all():
            continue
        Lv, Rv = V[inL], V[~inL]
        mask[Rv] = True
        on_sep = _rows_touching(rowptr, colind, Lv, mask)
        mask[Rv] = False
        nd.leaf, nd.ax, nd.t, nd.le = False, ax, float(t), le
        nd.sep = Lv[on_sep]
        nd.left = len(nodes)
        nodes.append(Node(nd.depth + 1, nd.bits * 2, Lv[~on_sep]))
        nd.right = len(nodes)
        nodes.append(Node(nd.depth + 1, nd.bits * 2 + 1, Rv))
        stack.extend([nd.right, nd.left])
    return nodes


def _descend(nodes, mi, verts, coords, depth):
    """Path bits below node mi for `verts`, by walking the stored cuts."""
    out = np.zeros(verts.size, dtype=np.int64)
    work = [(mi, np.arange(verts.size))]
    while work:
        m, sel = work.pop()
        nd = nodes[m]
        if nd.leaf or sel.size == 0:
            continue
        x = coords[verts[sel], nd.ax]
        go_left = (x <= nd.t) if nd.le else (x < nd.t)
        right = sel[~go_left]
        out[right] |= np.int64(1) << np.int64(depth - 1 - nd.depth)
        work.append((nd.left, sel[go_left]))
        work.append((nd.right, right))
    return out


def levels_and_paths(nodes, n, coords, depth):
    lvl = np.full(n, -1, dtype=np.int64)
    path = np.zeros(n, dtype=np.int64)
    for nd in nodes:
        if nd.leaf:
            lvl[nd.verts] = depth
            path[nd.verts] = np.int64(nd.bits) << np.int64(depth - nd.depth)
        else:
            S = nd.sep
            lvl[S] = nd.depth
            base = np.int64(nd.bits) << np.int64(depth - nd.depth)
            path[S] = base | _descend(nodes, nd.left, S, coords, depth)
    assert (lvl >= 0).all()
    return lvl, path


def _pairs_to_adj(pairs, nc):
    pairs = np.unique(pairs)
    i = pairs // nc
    j = pairs % nc
    split = np.searchsorted(i, np.arange(nc + 1))
    return [j[split[c]:split[c + 1]] for c in range(nc)], pairs


def _fill_pairs(adj, interiors, nc):
    out = []
    for s in interiors:
        nb = adj[s][adj[s] != s]
        if nb.size:
            a, b = np.meshgrid(nb, nb, indexing="ij")
            out.append((a * nc + b).ravel())
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def dsatur_colour(adj, interfaces, weight):
    """DSATUR colouring of the interface graph (see the module docstring).

    adj[p]: neighbours of p (interfaces among them); weight[p]: vertex count.
    Returns {p: colour}."""
    import heapq
    itf = set(interfaces)
    colour = {}
    seen = {p: set() for p in interfaces}
    heap = [(0, -int(weight[p]), p) for p in interfaces]
    heapq.heapify(heap)
    while heap:
        negsat, negw, p = heapq.heappop(heap)
        if p in colour or -negsat != len(seen[p]):
            continue                      # stale entry
        c = 0
        while c in seen[p]:
            c += 1
        colour[p] = c
        for q in adj[p]:
            q = int(q)
            if q in itf and q not in colour and c not in seen[q]:
                seen[q].add(c)
                heapq.heappush(heap, (-len(seen[q]), -int(weight[q]), q))
    return colour


def hop_distances(rowptr, colind, src):
    """Breadth-first hop distances from vertex src (n for unreachable vertices)."""
    n = rowptr.size - 1
    dist = np.full(n, n, dtype=np.int64)
    dist[src] = 0
    frontier = np.array([src], dtype=np.int64)
    d = 0
    while frontier.size:
        d += 1
        starts, ends = rowptr[frontier], rowptr[frontier + 1]
        nbr = np.concatenate([colind[a:b] for a, b in zip(starts, ends)]) if frontier.size else frontier
        nbr = np.unique(nbr)
        new = nbr[dist[nbr] == n]
        dist[new] = d
        frontier = new
    return dist


def graph_coords(rowptr, colind):
    """Landmark hop-distance coordinates (n x 3) of the coordinate-free reading."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    t = hop_distances(rowptr, colind, 0)
    l0 = int(np.argmax(t))                     # argmax: first (lowest) index of the maximum
    d0 = hop_distances(rowptr, colind, l0)
    l1 = int(np.argmax(d0))
    d1 = hop_distances(rowptr, colind, l1)
    l2 = int(np.argmax(np.minimum(d0, d1)))
    d2 = hop_distances(rowptr, colind, l2)
    return np.stack([d0, d1, d2], axis=1).astype(np.float64)


def analyze(rowptr, colind, coords, depth, skip=4):
    """Geometric ND plus the per-step cluster structure (see module docstring);
    coords None: the coordinate-free reading (landmark hop distances)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    if coords is None:
        coords = graph_coords(rowptr, colind)
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    D = int(depth)
    nodes = dissect(rowptr, colind, coords, D)
    lvl, path = levels_and_paths(nodes, n, coords, D)
    perm = np.lexsort((np.arange(n), path, D - lvl))
    plan = Plan(n, D, int(skip), lvl, path, perm, nodes)

    prev = None          # previous (finer) step
    prev_pairs = None
    for l in range(D, -1, -1):
        pre = path >> np.int64(D - l)
        alive = lvl <= l
        int_keys = np.unique(pre[lvl == l])
        itf_sel = lvl < l
        itf_codes, itf_nv = np.unique(lvl[itf_sel] * (np.int64(1) << np.int64(D + 1)) + pre[itf_sel],
                                      return_counts=True)
        keys = [(0, l, int(p)) for p in int_keys]
        keys += [(1, int(c >> (D + 1)), int(c & ((1 << (D + 1)) - 1))) for c in itf_codes]
        nI = len(int_keys)
        nc = len(keys)
        index = {k: i for i, k in enumerate(keys)}

        children = None
        verts = None
        if l == D:
            cid = np.full(n, -1, dtype=np.int64)
            cid[lvl == l] = np.searchsorted(int_keys, pre[lvl == l])
            code = lvl * (np.int64(1) << np.int64(D + 1)) + pre
            cid[itf_sel] = nI + np.searchsorted(itf_codes, code[itf_sel])
            order = np.lexsort((np.arange(n), cid))
            bounds = np.searchsorted(cid[order], np.arange(nc + 1))
            verts = [np.sort(order[bounds[c]:bounds[c + 1]]) for c in range(nc)]
            src = np.repeat(np.arange(n), np.diff(rowptr))
            pairs = cid[src] * nc + cid[colind]
            pairs = np.concatenate([pairs, np.arange(nc) * nc + np.arange(nc)])
        else:
            parent = np.full(prev.n_clusters, -1, dtype=np.int64)
            children = [[] for _ in range(nc)]
            for ci in range(prev.n_interior, prev.n_clusters):
                _, cl, cp = prev.keys[ci]
                key = (0, l, cp >> 1) if cl == l else (1, cl, cp >> 1)
                parent[ci] = index[key]
                children[parent[ci]].append(ci)
            pi = prev_pairs // prev.n_clusters
            pj = prev_pairs % prev.n_clusters
            keep = (parent[pi] >= 0) & (parent[pj] >= 0)
            pairs = parent[pi[keep]] * nc + parent[pj[keep]]
            pairs = np.concatenate([pairs, np.arange(nc) * nc + np.arange(nc)])
        adj, pairs = _pairs_to_adj(pairs, nc)
        fill = _fill_pairs(adj, range(nI), nc)
        if fill.size:
            adj, pairs = _pairs_to_adj(np.concatenate([pairs, fill]), nc)
        interfaces = list(range(nI, nc))
        itf_adj = [adj[p][adj[p] >= nI] for p in range(nc)]
        weight = {nI + i: int(c) for i, c in enumerate(itf_nv)}
        col = dsatur_colour(itf_adj, interfaces, weight)
        colour = np.full(nc, -1, dtype=np.int64)
        for p, c in col.items():
            colour[p] = c
        sparsified = 1 <= l <= D - plan.skip
        order = sorted(interfaces, key=lambda p: (colour[p], p))
        st = Step(l, keys, nI, adj, colour, sparsified, order, children, verts)
        plan.steps[l] = st
        prev, prev_pairs = st, pairs
    return plan


def check_plan(plan, rowptr, colind):
    """Structural invariants of the partition (raise AssertionError on failure)."""
    D = plan.depth
    n = plan.n
    st = plan.steps[D]
    seen = np.zeros(n, dtype=np.int64)
    for v in st.verts:
        seen[v] += 1
    assert (seen == 1).all(), "every vertex in exactly one step-depth cluster"
    for l, st in plan.steps.items():
        for s in range(st.n_interior):
            for t in st.adj[s]:
                assert t == s or t >= st.n_interior, f"interiors {s},{t} adjacent at step {l}"
        if st.children is not None:
            prev = plan.steps[l + 1]
            cnt = np.zeros(prev.n_clusters, dtype=np.int64)
            for ch in st.children:
                for c in ch:
                    cnt[c] += 1
            assert (cnt[:prev.n_interior] == 0).all()
            assert (cnt[prev.n_interior:] == 1).all(), "each interface maps to one parent"
        for p in st.order:
            for q in st.adj[p]:
                if q != p and q >= st.n_interior:
                    assert st.colour[p] != st.colour[q]
    # separators separate: no edge between a left subtree and the right subtree
    rowptr = np.asarray(rowptr)
    colind = np.asarray(colind)
    for nd in plan.nodes:
        if nd.leaf:
            continue
        L = plan.nodes[nd.left].verts
        R = plan.nodes[nd.right].verts
        mark = np.zeros(n, dtype=bool)
        mark[R] = True
        assert not _rows_touching(rowptr, colind.astype(np.int64), L, mark).any()
