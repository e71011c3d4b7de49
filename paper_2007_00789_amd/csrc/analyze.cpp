// Host symbolic analysis: geometric nested dissection, vertex levels and
// paths, clusters of every step, block adjacency with symbolic fill, greedy
// interface colouring, and the leaf-step panel layout.
//
// The paper's partition is algebraic and deferred to the base spaND paper
// (Sec. 3); this library uses a coordinate-bisection reading:
//  * a node at depth d with vertex set V is a leaf if d == depth, |V| <= 1 or
//    all coordinate extents are 0; otherwise it cuts the axis of largest
//    extent (lowest axis on ties) at t = x_axis of the element at |V|/2 of V
//    sorted by (x_axis, id); left = {x < t}, or {x <= t} when that is empty;
//    a node whose right side would be empty is a leaf;
//  * its separator is the set of left vertices with a neighbour on the right;
//    the left child holds the rest of the left side, the right child the right;
//  * paths: bit of depth e at position depth-1-e; separator vertices of a node
//    continue with bit 0 and then descend its left subtree along stored cuts;
//  * at step l the interiors are the vertices of level l grouped by path prefix,
//    the interfaces the vertices of level < l grouped by (level, prefix);
//  * clusters are adjacent if A couples them or if they border a common
//    interior eliminated at this or an earlier step; adjacency is inherited by
//    parents;
//  * interfaces are coloured greedily in canonical order and sparsified by
//    (colour, index) on the levels 1 <= l <= depth - skip (Alg. 2, Sec. 4).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace spand {

namespace {

struct Node {
  int depth = 0;
  int64_t bits = 0;
  std::vector<int32_t> verts;
  bool leaf = true;
  int ax = -1;
  double t = 0.0;
  bool le = false;
  int left = -1, right = -1;
  std::vector<int32_t> sep;
};

std::vector<Node> build_tree(const Plan& P, const double* coords, int dim) {
  const int D = P.depth;
  std::vector<Node> nodes(1);
  nodes[0].verts.resize(P.n);
  std::iota(nodes[0].verts.begin(), nodes[0].verts.end(), 0);
  std::vector<char> onR(P.n, 0);
  std::vector<int> stack{0};
  std::vector<double> lo(dim), hi(dim);
  while (!stack.empty()) {
    const int ni = stack.back();
    stack.pop_back();
    if (nodes[ni].depth == D || nodes[ni].verts.size() <= 1) continue;
    std::vector<int32_t> V = nodes[ni].verts;
    for (int a = 0; a < dim; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int32_t v : V)
      for (int a = 0; a < dim; ++a) {
        const double x = coords[(int64_t)v * dim + a];
        lo[a] = std::min(lo[a], x);
        hi[a] = std::max(hi[a], x);
      }
    int ax = 0;
    double best = hi[0] - lo[0];
    for (int a = 1; a < dim; ++a)
      if (hi[a] - lo[a] > best) { best = hi[a] - lo[a]; ax = a; }
    if (best == 0.0) continue;
    auto X = [&](int32_t v) { return coords[(int64_t)v * dim + ax]; };
    std::vector<int32_t> sorted = V;
    const size_t mid = V.size() / 2;
    std::nth_element(sorted.begin(), sorted.begin() + mid, sorted.end(), [&](int32_t a, int32_t b) {
      const double xa = X(a), xb = X(b);
      return xa < xb || (xa == xb && a < b);
    });
    const double t = X(sorted[mid]);
    bool le = false;
    size_t nl = 0;
    for (int32_t v : V) nl += X(v) < t;
    if (nl == 0) {
      le = true;
      for (int32_t v : V) nl += X(v) <= t;
    }
    if (nl == V.size()) continue;
    std::vector<int32_t> L, R;
    L.reserve(nl);
    R.reserve(V.size() - nl);
    for (int32_t v : V) {
      const bool left = le ? X(v) <= t : X(v) < t;
      (left ? L : R).push_back(v);
    }
    for (int32_t v : R) onR[v] = 1;
    std::vector<int32_t> S, Lrest;
    for (int32_t v : L) {
      bool touch = false;
      for (int64_t e = P.rowptr[v]; e < P.rowptr[v + 1] && !touch; ++e) touch = onR[P.colind[e]];
      (touch ? S : Lrest).push_back(v);
    }
    for (int32_t v : R) onR[v] = 0;
    Node ln, rn;
    ln.depth = rn.depth = nodes[ni].depth + 1;
    ln.bits = nodes[ni].bits * 2;
    rn.bits = nodes[ni].bits * 2 + 1;
    ln.verts = std::move(Lrest);
    rn.verts = std::move(R);
    const int li = (int)nodes.size();
    nodes.push_back(std::move(ln));
    nodes.push_back(std::move(rn));
    Node& nd = nodes[ni];
    nd.leaf = false;
    nd.ax = ax;
    nd.t = t;
    nd.le = le;
    nd.sep = std::move(S);
    nd.left = li;
    nd.right = li + 1;
    nd.verts.clear();
    nd.verts.shrink_to_fit();
    stack.push_back(li + 1);
    stack.push_back(li);
  }
  return nodes;
}

inline void sort_unique(std::vector<int64_t>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

// position of `target` in c's sorted adjacency list, or -1
int64_t adj_pos(const StepPlan& st, int c, int target) {
  const int32_t* b = st.adj.data() + st.adj_ptr[c];
  const int32_t* e = st.adj.data() + st.adj_ptr[c + 1];
  const int32_t* it = std::lower_bound(b, e, target);
  if (it == e || *it != target) return -1;
  return st.adj_ptr[c] + (it - b);
}

// reverse adjacency positions, Schur targets and merge copies of step l
void build_numeric_lists(Plan& P, int l) {
  StepPlan& st = P.steps[l];
  const int nI = st.nI, nc = st.nc;
  st.adj_rev.assign(st.adj.size(), -1);
  for (int c = 0; c < nc; ++c)
    for (int64_t e = st.adj_ptr[c]; e < st.adj_ptr[c + 1]; ++e)
      st.adj_rev[e] = adj_pos(st, st.adj[e], c);
  st.schur.clear();
  st.schur_terms.clear();
  for (int w1 = nI; w1 < nc; ++w1) {
    const int64_t b1 = st.adj_ptr[w1], e1 = st.adj_ptr[w1 + 1];
    int64_t i1end = b1;
    while (i1end < e1 && st.adj[i1end] < nI) ++i1end;
    if (i1end == b1) continue;  // no interior neighbour
    for (int64_t e = i1end; e < e1; ++e) {
      const int w2 = st.adj[e];
      if (w2 < w1) continue;
      const int64_t b2 = st.adj_ptr[w2], e2 = st.adj_ptr[w2 + 1];
      const int64_t t0 = (int64_t)st.schur_terms.size();
      int64_t x = b1, y = b2;
      while (x < i1end && y < e2 && st.adj[y] < nI) {
        if (st.adj[x] < st.adj[y]) ++x;
        else if (st.adj[y] < st.adj[x]) ++y;
        else {
          st.schur_terms.push_back({st.adj[x], 0, st.adj_rev[x], st.adj_rev[y]});
          ++x;
          ++y;
        }
      }
      if ((int64_t)st.schur_terms.size() > t0)
        st.schur.push_back({w1, w2, e, t0, (int64_t)st.schur_terms.size()});
    }
  }
  st.merge.clear();
  if (l == 0) return;
  const StepPlan& nx = P.steps[l - 1];
  for (int Pc = 0; Pc < nx.nc; ++Pc)
    for (int64_t e = nx.adj_ptr[Pc]; e < nx.adj_ptr[Pc + 1]; ++e) {
      const int Q = nx.adj[e];
      for (int64_t a = nx.child_ptr[Pc]; a < nx.child_ptr[Pc + 1]; ++a) {
        const int ci = nx.child[a];
        for (int64_t b = nx.child_ptr[Q]; b < nx.child_ptr[Q + 1]; ++b) {
          const int cj = nx.child[b];
          const int64_t ee = adj_pos(st, ci, cj);
          if (ee >= 0) st.merge.push_back({Pc, ci, cj, 0, e, ee});
        }
      }
    }
}

}  // namespace

void analyze_plan(Plan& P, const int64_t* rowptr, const int32_t* colind, const double* coords,
                  int dim, int depth, int skip) {
  const int64_t n = P.n;
  P.dim = dim;
  P.depth = depth;
  P.skip = skip;
  P.rowptr.assign(rowptr, rowptr + n + 1);
  P.nnz = P.rowptr[n];
  P.colind.assign(colind, colind + P.nnz);
  const int D = depth;

  // pattern symmetry: sort each row's columns and look every entry up
  {
    std::vector<int32_t> srt(P.colind);
    for (int64_t i = 0; i < n; ++i) {
      if (P.rowptr[i + 1] < P.rowptr[i]) throw Error(SPAND_E_INVALID, "rowptr not monotone");
      std::sort(srt.begin() + P.rowptr[i], srt.begin() + P.rowptr[i + 1]);
    }
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
        const int32_t j = srt[e];
        if (j < 0 || j >= n) throw Error(SPAND_E_INVALID, "column index out of range");
        if (!std::binary_search(srt.begin() + P.rowptr[j], srt.begin() + P.rowptr[j + 1], (int32_t)i))
          throw Error(SPAND_E_NOT_SYMMETRIC, "pattern not symmetric at row " + std::to_string(i) +
                                                 ", column " + std::to_string(j));
      }
  }

  std::vector<Node> nodes = build_tree(P, coords, dim);

  // levels and paths
  P.lvl.assign(n, -1);
  P.path.assign(n, 0);
  for (const Node& nd : nodes) {
    const int64_t base = nd.bits << (D - nd.depth);
    if (nd.leaf) {
      for (int32_t v : nd.verts) { P.lvl[v] = D; P.path[v] = base; }
      continue;
    }
    for (int32_t v : nd.sep) {
      int64_t bits = 0;
      int m = nd.left;
      while (!nodes[m].leaf) {
        const Node& M = nodes[m];
        const double x = coords[(int64_t)v * dim + M.ax];
        const bool goleft = M.le ? x <= M.t : x < M.t;
        if (!goleft) bits |= int64_t(1) << (D - 1 - M.depth);
        m = goleft ? M.left : M.right;
      }
      P.lvl[v] = nd.depth;
      P.path[v] = base | bits;
    }
  }
  P.perm.resize(n);
  std::iota(P.perm.begin(), P.perm.end(), 0);
  std::sort(P.perm.begin(), P.perm.end(), [&](int64_t a, int64_t b) {
    const int la = D - P.lvl[a], lb = D - P.lvl[b];
    if (la != lb) return la < lb;
    if (P.path[a] != P.path[b]) return P.path[a] < P.path[b];
    return a < b;
  });

  // clusters, adjacency and colours of every step
  P.steps.assign(D + 1, StepPlan());
  std::vector<int64_t> prev_pairs;
  const int64_t SH = int64_t(1) << (D + 1);
  for (int l = D; l >= 0; --l) {
    StepPlan& st = P.steps[l];
    st.l = l;
    std::vector<int64_t> ikeys, fkeys;  // interior prefixes; interface codes lvl*SH + prefix
    for (int64_t v = 0; v < n; ++v) {
      const int64_t pre = P.path[v] >> (D - l);
      if (P.lvl[v] == l) ikeys.push_back(pre);
      else if (P.lvl[v] < l) fkeys.push_back(P.lvl[v] * SH + pre);
    }
    sort_unique(ikeys);
    sort_unique(fkeys);
    st.nI = (int)ikeys.size();
    st.nc = st.nI + (int)fkeys.size();
    const int nc = st.nc;
    st.key_lvl.resize(nc);
    st.key_prefix.resize(nc);
    for (int i = 0; i < st.nI; ++i) { st.key_lvl[i] = l; st.key_prefix[i] = ikeys[i]; }
    for (size_t i = 0; i < fkeys.size(); ++i) {
      st.key_lvl[st.nI + i] = fkeys[i] / SH;
      st.key_prefix[st.nI + i] = fkeys[i] % SH;
    }
    auto find_interior = [&](int64_t pre) {
      auto it = std::lower_bound(ikeys.begin(), ikeys.end(), pre);
      return (int)(it - ikeys.begin());
    };
    auto find_interface = [&](int64_t code) {
      auto it = std::lower_bound(fkeys.begin(), fkeys.end(), code);
      return st.nI + (int)(it - fkeys.begin());
    };

    std::vector<int64_t> pairs;
    if (l == D) {
      std::vector<int32_t> cid(n);
      for (int64_t v = 0; v < n; ++v) {
        const int64_t pre = P.path[v] >> (D - l);
        cid[v] = P.lvl[v] == l ? find_interior(pre) : find_interface(P.lvl[v] * SH + pre);
      }
      st.vert_ptr.assign(nc + 1, 0);
      for (int64_t v = 0; v < n; ++v) st.vert_ptr[cid[v] + 1]++;
      for (int c = 0; c < nc; ++c) st.vert_ptr[c + 1] += st.vert_ptr[c];
      st.verts.resize(n);
      std::vector<int64_t> fillp(st.vert_ptr.begin(), st.vert_ptr.end() - 1);
      for (int64_t v = 0; v < n; ++v) st.verts[fillp[cid[v]]++] = (int32_t)v;  // ascending ids
      pairs.reserve(P.nnz + nc);
      for (int64_t v = 0; v < n; ++v)
        for (int64_t e = P.rowptr[v]; e < P.rowptr[v + 1]; ++e)
          pairs.push_back((int64_t)cid[v] * nc + cid[P.colind[e]]);
    } else {
      const StepPlan& pv = P.steps[l + 1];
      StepPlan& pvm = P.steps[l + 1];
      pvm.parent.assign(pv.nc, -1);
      st.child_ptr.assign(nc + 1, 0);
      std::vector<std::vector<int32_t>> ch(nc);
      for (int c = pv.nI; c < pv.nc; ++c) {
        const int64_t cl = pv.key_lvl[c], cp = pv.key_prefix[c] >> 1;
        const int par = cl == l ? find_interior(cp) : find_interface(cl * SH + cp);
        pvm.parent[c] = par;
        ch[par].push_back(c);
      }
      for (int c = 0; c < nc; ++c) st.child_ptr[c + 1] = st.child_ptr[c] + ch[c].size();
      st.child.reserve(st.child_ptr[nc]);
      for (int c = 0; c < nc; ++c) st.child.insert(st.child.end(), ch[c].begin(), ch[c].end());
      const int64_t pnc = pv.nc;
      pairs.reserve(prev_pairs.size() + nc);
      for (int64_t code : prev_pairs) {
        const int32_t a = pvm.parent[code / pnc], b = pvm.parent[code % pnc];
        if (a >= 0 && b >= 0) pairs.push_back((int64_t)a * nc + b);
      }
    }
    for (int c = 0; c < nc; ++c) pairs.push_back((int64_t)c * nc + c);
    sort_unique(pairs);
    // fill from the interiors of this step
    {
      std::vector<int64_t> fill;
      auto begin_of = [&](int c) {
        return std::lower_bound(pairs.begin(), pairs.end(), (int64_t)c * nc) - pairs.begin();
      };
      for (int s = 0; s < st.nI; ++s) {
        std::vector<int32_t> nb;
        for (int64_t e = begin_of(s); e < (int64_t)pairs.size() && pairs[e] / nc == s; ++e)
          if (pairs[e] % nc != s) nb.push_back((int32_t)(pairs[e] % nc));
        for (int32_t a : nb)
          for (int32_t b : nb) fill.push_back((int64_t)a * nc + b);
      }
      if (!fill.empty()) {
        pairs.insert(pairs.end(), fill.begin(), fill.end());
        sort_unique(pairs);
      }
    }
    st.adj_ptr.assign(nc + 1, 0);
    st.adj.resize(pairs.size());
    for (size_t e = 0; e < pairs.size(); ++e) {
      st.adj_ptr[pairs[e] / nc + 1]++;
      st.adj[e] = (int32_t)(pairs[e] % nc);
    }
    for (int c = 0; c < nc; ++c) st.adj_ptr[c + 1] += st.adj_ptr[c];
    // greedy colouring of the interface graph in canonical order
    st.colour.assign(nc, -1);
    st.ncolours = 0;
    std::vector<char> used;
    for (int p = st.nI; p < nc; ++p) {
      used.assign(st.ncolours + 2, 0);
      for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
        const int q = st.adj[e];
        if (q >= st.nI && q < p) used[st.colour[q]] = 1;
      }
      int c = 0;
      while (used[c]) ++c;
      st.colour[p] = c;
      st.ncolours = std::max(st.ncolours, c + 1);
    }
    st.order.clear();
    for (int p = st.nI; p < nc; ++p) st.order.push_back(p);
    std::stable_sort(st.order.begin(), st.order.end(),
                     [&](int a, int b) { return st.colour[a] < st.colour[b]; });
    st.sparsified = l >= 1 && l <= D - skip;
    prev_pairs.swap(pairs);
  }
  P.steps[0].parent.assign(P.steps[0].nc, -1);
  for (int l = 0; l <= D; ++l)
    if (P.steps[l].parent.empty()) P.steps[l].parent.assign(P.steps[l].nc, -1);
  for (int l = 0; l <= D; ++l) build_numeric_lists(P, l);
}

void merge_plans(Plan& M, std::vector<Plan>& parts, int skip) {
  const int np = (int)parts.size();
  int D = 0;
  for (const Plan& q : parts) D = std::max(D, q.depth);
  M.depth = D;
  M.skip = skip;
  M.dim = parts.empty() ? 0 : parts[0].dim;
  std::vector<int64_t> voff(np + 1, 0), eoff(np + 1, 0);
  for (int i = 0; i < np; ++i) {
    voff[i + 1] = voff[i] + parts[i].n;
    eoff[i + 1] = eoff[i] + parts[i].nnz;
  }
  M.n = voff[np];
  M.nnz = eoff[np];
  if (M.n >= (int64_t(1) << 31)) throw Error(SPAND_E_LIMIT, "batch larger than 2^31 rows");
  M.rowptr.assign(1, 0);
  M.colind.clear();
  M.lvl.clear();
  M.path.clear();
  M.perm.clear();
  M.seg_off = voff;
  M.seg_id.assign(M.n, 0);
  for (int i = 0; i < np; ++i) {
    const Plan& q = parts[i];
    const int shift = D - q.depth;
    for (int64_t v = 0; v < q.n; ++v) {
      M.rowptr.push_back(eoff[i] + q.rowptr[v + 1]);
      M.lvl.push_back(q.lvl[v] + shift);
      M.path.push_back(q.path[v]);
      M.perm.push_back(q.perm[v] + voff[i]);
      M.seg_id[voff[i] + v] = i;
    }
    for (int64_t e = 0; e < q.nnz; ++e) M.colind.push_back((int32_t)(q.colind[e] + voff[i]));
  }
  // cluster maps of every merged step: interiors of all problems first (in
  // problem order), then their interfaces
  M.steps.assign(D + 1, StepPlan());
  std::vector<std::vector<int32_t>> ioff(D + 1, std::vector<int32_t>(np, 0)),
      foff(D + 1, std::vector<int32_t>(np, 0));
  auto own = [&](int i, int lm) { return lm - (D - parts[i].depth); };   // problem step
  for (int lm = 0; lm <= D; ++lm) {
    StepPlan& S = M.steps[lm];
    S.l = lm;
    int nI = 0, nF = 0;
    for (int i = 0; i < np; ++i) {
      const int l = own(i, lm);
      ioff[lm][i] = nI;
      foff[lm][i] = nF;
      if (l < 0) continue;
      nI += parts[i].steps[l].nI;
      nF += parts[i].steps[l].nc - parts[i].steps[l].nI;
    }
    S.nI = nI;
    S.nc = nI + nF;
    S.sparsified = lm >= 1 && lm <= D - skip;
  }
  auto map = [&](int lm, int i, int c) {
    const StepPlan& q = parts[i].steps[own(i, lm)];
    return c < q.nI ? ioff[lm][i] + c : M.steps[lm].nI + foff[lm][i] + (c - q.nI);
  };
  for (int lm = 0; lm <= D; ++lm) {
    StepPlan& S = M.steps[lm];
    const int nc = S.nc;
    S.key_lvl.assign(nc, 0);
    S.key_prefix.assign(nc, 0);
    S.colour.assign(nc, -1);
    S.parent.assign(nc, -1);
    std::vector<std::pair<int, int>> owner(nc);
    for (int i = 0; i < np; ++i) {
      const int l = own(i, lm);
      if (l < 0) continue;
      const StepPlan& q = parts[i].steps[l];
      for (int c = 0; c < q.nc; ++c) {
        const int x = map(lm, i, c);
        owner[x] = {i, c};
        S.key_lvl[x] = q.key_lvl[c] + (D - parts[i].depth);
        S.key_prefix[x] = q.key_prefix[c];
        S.colour[x] = q.colour[c];
        if (lm > 0 && !q.parent.empty() && q.parent[c] >= 0 && l > 0)
          S.parent[x] = map(lm - 1, i, q.parent[c]);
      }
    }
    S.adj_ptr.assign(nc + 1, 0);
    S.adj.clear();
    for (int x = 0; x < nc; ++x) {
      const auto [i, c] = owner[x];
      const StepPlan& q = parts[i].steps[own(i, lm)];
      for (int64_t e = q.adj_ptr[c]; e < q.adj_ptr[c + 1]; ++e) S.adj.push_back(map(lm, i, q.adj[e]));
      S.adj_ptr[x + 1] = (int64_t)S.adj.size();
    }
    S.ncolours = 0;
    for (int x = S.nI; x < nc; ++x) S.ncolours = std::max(S.ncolours, S.colour[x] + 1);
    S.order.clear();
    for (int x = S.nI; x < nc; ++x) S.order.push_back(x);
    std::stable_sort(S.order.begin(), S.order.end(),
                     [&](int a, int b) { return S.colour[a] < S.colour[b]; });
    if (lm < D) {   // children in step lm + 1
      S.child_ptr.assign(nc + 1, 0);
      S.child.clear();
      for (int x = 0; x < nc; ++x) {
        const auto [i, c] = owner[x];
        const StepPlan& q = parts[i].steps[own(i, lm)];
        if (!q.child_ptr.empty())
          for (int64_t e = q.child_ptr[c]; e < q.child_ptr[c + 1]; ++e)
            S.child.push_back(map(lm + 1, i, q.child[e]));
        S.child_ptr[x + 1] = (int64_t)S.child.size();
      }
    } else {        // leaf step: vertices of every cluster
      S.vert_ptr.assign(nc + 1, 0);
      S.verts.clear();
      for (int x = 0; x < nc; ++x) {
        const auto [i, c] = owner[x];
        const StepPlan& q = parts[i].steps[parts[i].depth];
        for (int64_t e = q.vert_ptr[c]; e < q.vert_ptr[c + 1]; ++e)
          S.verts.push_back((int32_t)(q.verts[e] + voff[i]));
        S.vert_ptr[x + 1] = (int64_t)S.verts.size();
      }
    }
  }
  for (int lm = 0; lm <= D; ++lm) build_numeric_lists(M, lm);
}

void build_leaf_map(Plan& P) {
  const int64_t n = P.n;
  const StepPlan& st0 = P.steps[P.depth];
  std::vector<int32_t> sizes(st0.nc), cid(n), loc(n);
  for (int c = 0; c < st0.nc; ++c) {
    sizes[c] = (int32_t)(st0.vert_ptr[c + 1] - st0.vert_ptr[c]);
    for (int64_t e = st0.vert_ptr[c]; e < st0.vert_ptr[c + 1]; ++e) {
      cid[st0.verts[e]] = c;
      loc[st0.verts[e]] = (int32_t)(e - st0.vert_ptr[c]);
    }
  }
  PanelLayout lay = make_layout(st0, sizes);
  std::vector<int64_t> dest(P.nnz);
  for (int64_t v = 0; v < n; ++v) {
    const int c = cid[v];
    for (int64_t e = P.rowptr[v]; e < P.rowptr[v + 1]; ++e) {
      const int32_t u = P.colind[e];
      const int c2 = cid[u];
      const int32_t* b = st0.adj.data() + st0.adj_ptr[c];
      const int32_t* en = st0.adj.data() + st0.adj_ptr[c + 1];
      const int64_t ee = st0.adj_ptr[c] + (std::lower_bound(b, en, c2) - b);
      dest[e] = lay.off[c] + (lay.coff[ee] + loc[u]) * sizes[c] + loc[v];
    }
  }
  P.leaf_panel_elems = lay.total;
  P.leaf_dest = std::move(dest);
  if (P.seg_off.empty()) P.seg_off = {0, n};
}

PanelLayout make_layout(const StepPlan& st, const std::vector<int32_t>& sizes) {
  PanelLayout L;
  L.n = sizes;
  L.off.resize(st.nc);
  L.width.resize(st.nc);
  L.coff.resize(st.adj.size());
  int64_t off = 0;
  for (int c = 0; c < st.nc; ++c) {
    int64_t w = 0;
    for (int64_t e = st.adj_ptr[c]; e < st.adj_ptr[c + 1]; ++e) {
      L.coff[e] = w;
      w += sizes[st.adj[e]];
    }
    L.width[c] = w;
    L.off[c] = off;
    off += (int64_t)sizes[c] * w;
    off = (off + 1) & ~int64_t(1);  // 16-byte alignment of every panel
  }
  L.total = off;
  return L;
}

}  // namespace spand
