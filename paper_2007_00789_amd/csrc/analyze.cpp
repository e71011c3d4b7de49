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
//  * interfaces are coloured by DSATUR (saturation, then vertex count, then
//    index) and sparsified by (colour, index) on the levels
//    1 <= l <= depth - skip (Alg. 2, Sec. 4).
#include <algorithm>
#include <tuple>
#include <queue>
#include <atomic>
#include <cmath>
#include <memory>
#include <numeric>
#include <thread>

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

// Runs f(i) for 0 <= i < count on up to nth host threads.
template <class F>
void parallel_for(int count, int nth, const F& f) {
  std::atomic<int> next{0};
  auto run = [&] {
    for (int i; (i = next.fetch_add(1)) < count;) f(i);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < std::min(nth, count); ++t) pool.emplace_back(run);
  run();
  for (auto& t : pool) t.join();
}

int host_threads(int64_t work) {
  return work >= (1 << 17) ? std::min(16, (int)std::max(1u, std::thread::hardware_concurrency())) : 1;
}

// Marks of the right side of the node being split: a vertex belongs to it if
// its stamp is the node's own (stamps are unique, so nodes split concurrently
// on disjoint vertex sets never see each other's marks).
struct SideMarks {
  std::unique_ptr<std::atomic<int32_t>[]> owner;
  std::atomic<int32_t> stamps{0};
  explicit SideMarks(int64_t n) : owner(new std::atomic<int32_t>[n]) {
    for (int64_t i = 0; i < n; ++i) owner[i].store(0, std::memory_order_relaxed);
  }
};

// Splits node nd into the children ln and rn (their indices are set by the
// caller), unless it is a leaf.
bool split_node(Node& nd, Node& ln, Node& rn, const Plan& P, const double* coords, int dim,
                SideMarks& marks) {
  if (nd.depth == P.depth || nd.verts.size() <= 1) return false;
  std::atomic<int32_t>* owner = marks.owner.get();
  std::atomic<int32_t>& stamps = marks.stamps;
  double lo[3], hi[3];
  // the order of a node's vertex list carries no meaning: it is partitioned
  // in place (the cut and the separator depend on the vertex set only)
  std::vector<int32_t>& V = nd.verts;
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
  if (best == 0.0) return false;
  auto X = [&](int32_t v) { return coords[(int64_t)v * dim + ax]; };
  const size_t mid = V.size() / 2;
  std::nth_element(V.begin(), V.begin() + mid, V.end(), [&](int32_t a, int32_t b) {
    const double xa = X(a), xb = X(b);
    return xa < xb || (xa == xb && a < b);
  });
  const double t = X(V[mid]);
  bool le = false;
  size_t nl = 0;
  for (int32_t v : V) nl += X(v) < t;
  if (nl == 0) {
    le = true;
    for (int32_t v : V) nl += X(v) <= t;
  }
  if (nl == V.size()) return false;
  std::vector<int32_t> L, R;
  L.reserve(nl);
  R.reserve(V.size() - nl);
  for (int32_t v : V) {
    const bool left = le ? X(v) <= t : X(v) < t;
    (left ? L : R).push_back(v);
  }
  std::vector<int32_t>().swap(V);
  const int32_t stamp = stamps.fetch_add(1, std::memory_order_relaxed) + 1;
  for (int32_t v : R) owner[v].store(stamp, std::memory_order_relaxed);
  std::vector<int32_t> S, Lrest;
  for (int32_t v : L) {
    bool touch = false;
    for (int64_t e = P.rowptr[v]; e < P.rowptr[v + 1] && !touch; ++e)
      touch = owner[P.colind[e]].load(std::memory_order_relaxed) == stamp;
    (touch ? S : Lrest).push_back(v);
  }
  ln.depth = rn.depth = nd.depth + 1;
  ln.bits = nd.bits * 2;
  rn.bits = nd.bits * 2 + 1;
  ln.verts = std::move(Lrest);
  rn.verts = std::move(R);
  nd.leaf = false;
  nd.ax = ax;
  nd.t = t;
  nd.le = le;
  nd.sep = std::move(S);
  return true;
}

// Appends the children of node ni and links them.
void attach(std::vector<Node>& nodes, int ni, Node& ln, Node& rn) {
  const int li = (int)nodes.size();
  nodes.push_back(std::move(ln));
  nodes.push_back(std::move(rn));
  nodes[ni].left = li;
  nodes[ni].right = li + 1;
}

void grow(std::vector<Node>& nodes, int root, const Plan& P, const double* coords, int dim,
          SideMarks& marks) {
  std::vector<int> stack{root};
  while (!stack.empty()) {
    const int ni = stack.back();
    stack.pop_back();
    Node ln, rn;
    if (split_node(nodes[ni], ln, rn, P, coords, dim, marks)) {
      attach(nodes, ni, ln, rn);
      stack.push_back(nodes[ni].right);
      stack.push_back(nodes[ni].left);
    }
  }
}

// The node tree: the top levels on this thread, breadth first, until there
// are enough independent subtrees; those are grown on up to 16 host threads
// into lists of their own and spliced in.  Node indices differ from a serial
// build, which nothing depends on: every node carries its own depth and bits.
std::vector<Node> build_tree(const Plan& P, const double* coords, int dim) {
  std::vector<Node> nodes(1);
  nodes[0].verts.resize(P.n);
  std::iota(nodes[0].verts.begin(), nodes[0].verts.end(), 0);
  SideMarks marks(P.n);
  const int nth = host_threads(P.n);
  if (nth == 1) {
    grow(nodes, 0, P, coords, dim, marks);
    return nodes;
  }
  // the top levels: the nodes of one level are split concurrently
  std::vector<int> frontier{0};
  while (!frontier.empty() && (int)frontier.size() < 4 * nth) {
    const int nf = (int)frontier.size();
    std::vector<Node> kids(2 * (size_t)nf);
    std::vector<char> split(nf, 0);
    parallel_for(nf, nth, [&](int i) {
      split[i] = split_node(nodes[frontier[i]], kids[2 * i], kids[2 * i + 1], P, coords, dim, marks);
    });
    std::vector<int> next;
    for (int i = 0; i < nf; ++i)
      if (split[i]) {
        attach(nodes, frontier[i], kids[2 * i], kids[2 * i + 1]);
        next.push_back(nodes[frontier[i]].left);
        next.push_back(nodes[frontier[i]].right);
      }
    frontier.swap(next);
  }
  // the subtrees below, each into a node list of its own
  const int nf = (int)frontier.size();
  std::vector<std::vector<Node>> sub(nf);
  for (int i = 0; i < nf; ++i) sub[i].push_back(std::move(nodes[frontier[i]]));
  parallel_for(nf, nth, [&](int i) { grow(sub[i], 0, P, coords, dim, marks); });
  for (int i = 0; i < nf; ++i) {
    const int base = (int)nodes.size() - 1;
    auto map = [&](int j) { return j == 0 ? frontier[i] : base + j; };
    for (Node& nd : sub[i])
      if (!nd.leaf) {
        nd.left = map(nd.left);
        nd.right = map(nd.right);
      }
    nodes[frontier[i]] = std::move(sub[i][0]);
    for (size_t j = 1; j < sub[i].size(); ++j) nodes.push_back(std::move(sub[i][j]));
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
    for (int64_t i = 0; i < n; ++i)
      if (P.rowptr[i + 1] < P.rowptr[i]) throw Error(SPAND_E_INVALID, "rowptr not monotone");
    for (int64_t e = 0; e < P.nnz; ++e)
      if (P.colind[e] < 0 || P.colind[e] >= n) throw Error(SPAND_E_INVALID, "column index out of range");
    std::vector<int32_t> srt(P.colind);
    // rows in chunks on host threads; the first asymmetric entry (lowest row)
    // is reported
    const int64_t chunk = 1 << 14;
    const int nchunk = (int)((n + chunk - 1) / chunk);
    const int nth = host_threads(P.nnz);
    parallel_for(nchunk, nth, [&](int k) {
      for (int64_t i = k * chunk; i < std::min(n, (k + 1) * chunk); ++i)
        std::sort(srt.begin() + P.rowptr[i], srt.begin() + P.rowptr[i + 1]);
    });
    std::vector<int64_t> bad(nchunk, -1);
    parallel_for(nchunk, nth, [&](int k) {
      for (int64_t i = k * chunk; i < std::min(n, (k + 1) * chunk) && bad[k] < 0; ++i)
        for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
          const int32_t j = srt[e];
          if (!std::binary_search(srt.begin() + P.rowptr[j], srt.begin() + P.rowptr[j + 1], (int32_t)i)) {
            bad[k] = e;
            break;
          }
        }
    });
    for (int k = 0; k < nchunk; ++k)
      if (bad[k] >= 0) {
        const int64_t e = bad[k];
        const int64_t i = std::upper_bound(P.rowptr.begin(), P.rowptr.end(), e) - P.rowptr.begin() - 1;
        throw Error(SPAND_E_NOT_SYMMETRIC, "pattern not symmetric at row " + std::to_string(i) +
                                               ", column " + std::to_string(srt[e]));
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
  // elimination order by (D - lvl, path, id): (D - lvl) * 2^(D+1) + path packs
  // the first two into one key (depth <= 40 keeps it below 2^47)
  {
    struct KV {
      uint64_t k;
      int64_t v;
      bool operator<(const KV& o) const { return k < o.k || (k == o.k && v < o.v); }
    };
    std::vector<KV> kv(n);
    for (int64_t v = 0; v < n; ++v)
      kv[v] = {((uint64_t)(D - P.lvl[v]) << (D + 1)) | (uint64_t)P.path[v], v};
    std::sort(kv.begin(), kv.end());
    P.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) P.perm[i] = kv[i].v;
  }

  // clusters, adjacency and colours of every step
  P.steps.assign(D + 1, StepPlan());
  const int64_t SH = int64_t(1) << (D + 1);
  std::vector<int32_t> mark;
  std::vector<int64_t> nv, nv_prev;   // vertices of A in each cluster (this step, the finer one)
  for (int l = D; l >= 0; --l) {
    StepPlan& st = P.steps[l];
    st.l = l;
    // cluster keys: interior prefixes, interface codes lvl * SH + prefix.  At
    // the leaf step from the vertices; above it from the interfaces of step
    // l + 1, which hold exactly the vertices of level < l + 1
    std::vector<int64_t> ikeys, fkeys;
    if (l == D) {
      for (int64_t v = 0; v < n; ++v) {
        if (P.lvl[v] == l) ikeys.push_back(P.path[v]);
        else fkeys.push_back(P.lvl[v] * SH + P.path[v]);
      }
    } else {
      const StepPlan& pv = P.steps[l + 1];
      for (int c = pv.nI; c < pv.nc; ++c) {
        const int64_t cl = pv.key_lvl[c], cp = pv.key_prefix[c] >> 1;
        if (cl == l) ikeys.push_back(cp);
        else fkeys.push_back(cl * SH + cp);
      }
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

    // adjacency before this step's fill (sorted lists, self included): at the
    // leaf step the clusters A couples; above it the parents of adjacent
    // interfaces of step l + 1
    std::vector<int64_t> ptr(nc + 1, 0);
    std::vector<int32_t> lst;
    mark.assign(nc, -1);
    if (l == D) {
      std::vector<int32_t> cid(n);
      for (int64_t v = 0; v < n; ++v)
        cid[v] = P.lvl[v] == l ? find_interior(P.path[v]) : find_interface(P.lvl[v] * SH + P.path[v]);
      st.vert_ptr.assign(nc + 1, 0);
      for (int64_t v = 0; v < n; ++v) st.vert_ptr[cid[v] + 1]++;
      for (int c = 0; c < nc; ++c) st.vert_ptr[c + 1] += st.vert_ptr[c];
      st.verts.resize(n);
      std::vector<int64_t> fillp(st.vert_ptr.begin(), st.vert_ptr.end() - 1);
      for (int64_t v = 0; v < n; ++v) st.verts[fillp[cid[v]]++] = (int32_t)v;  // ascending ids
      for (int c = 0; c < nc; ++c) {
        const size_t b0 = lst.size();
        mark[c] = c;
        lst.push_back(c);
        for (int64_t i = st.vert_ptr[c]; i < st.vert_ptr[c + 1]; ++i) {
          const int32_t v = st.verts[i];
          for (int64_t e = P.rowptr[v]; e < P.rowptr[v + 1]; ++e) {
            const int32_t q = cid[P.colind[e]];
            if (mark[q] != c) {
              mark[q] = c;
              lst.push_back(q);
            }
          }
        }
        std::sort(lst.begin() + b0, lst.end());
        ptr[c + 1] = (int64_t)lst.size();
      }
    } else {
      StepPlan& pv = P.steps[l + 1];
      pv.parent.assign(pv.nc, -1);
      st.child_ptr.assign(nc + 1, 0);
      std::vector<std::vector<int32_t>> ch(nc);
      for (int c = pv.nI; c < pv.nc; ++c) {
        const int64_t cl = pv.key_lvl[c], cp = pv.key_prefix[c] >> 1;
        const int par = cl == l ? find_interior(cp) : find_interface(cl * SH + cp);
        pv.parent[c] = par;
        ch[par].push_back(c);
      }
      for (int c = 0; c < nc; ++c) st.child_ptr[c + 1] = st.child_ptr[c] + ch[c].size();
      st.child.reserve(st.child_ptr[nc]);
      for (int c = 0; c < nc; ++c) st.child.insert(st.child.end(), ch[c].begin(), ch[c].end());
      for (int c = 0; c < nc; ++c) {
        const size_t b0 = lst.size();
        mark[c] = c;
        lst.push_back(c);
        for (int64_t a = st.child_ptr[c]; a < st.child_ptr[c + 1]; ++a) {
          const int x = st.child[a];
          for (int64_t e = pv.adj_ptr[x]; e < pv.adj_ptr[x + 1]; ++e) {
            const int32_t q = pv.parent[pv.adj[e]];
            if (q >= 0 && mark[q] != c) {
              mark[q] = c;
              lst.push_back(q);
            }
          }
        }
        std::sort(lst.begin() + b0, lst.end());
        ptr[c + 1] = (int64_t)lst.size();
      }
    }
    // fill from the interiors of this step: two clusters that border a common
    // interior s become adjacent.  The lists are symmetric, so cluster a gains
    // the neighbours of every interior s != a in its own list.
    st.adj_ptr.assign(nc + 1, 0);
    st.adj.clear();
    st.adj.reserve(lst.size());
    mark.assign(nc, -1);
    for (int a = 0; a < nc; ++a) {
      const size_t b0 = st.adj.size();
      bool grown = false;
      for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) {
        mark[lst[e]] = a;
        st.adj.push_back(lst[e]);
      }
      for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) {
        const int32_t s = lst[e];
        if (s >= st.nI || s == a) continue;
        for (int64_t f = ptr[s]; f < ptr[s + 1]; ++f) {
          const int32_t b = lst[f];
          if (b != s && mark[b] != a) {
            mark[b] = a;
            st.adj.push_back(b);
            grown = true;
          }
        }
      }
      if (grown) std::sort(st.adj.begin() + b0, st.adj.end());
      st.adj_ptr[a + 1] = (int64_t)st.adj.size();
    }
    // vertices of A per cluster: at the leaf step counted, above it summed
    // over the children
    nv.assign(nc, 0);
    if (l == D) {
      for (int c = 0; c < nc; ++c) nv[c] = st.vert_ptr[c + 1] - st.vert_ptr[c];
    } else {
      for (int c = 0; c < nc; ++c)
        for (int64_t a = st.child_ptr[c]; a < st.child_ptr[c + 1]; ++a) nv[c] += nv_prev[st.child[a]];
    }
    // DSATUR colouring of the interface graph: the uncoloured interface with
    // the most distinct colours among its coloured neighbours goes next (ties:
    // more vertices of A, then the lower index) and takes the smallest colour
    // none of them has
    st.colour.assign(nc, -1);
    st.ncolours = 0;
    {
      std::vector<std::vector<int32_t>> seen(nc);   // distinct neighbour colours, ascending
      using Key = std::tuple<int, int64_t, int>;    // (-saturation, -vertices, index)
      std::priority_queue<Key, std::vector<Key>, std::greater<Key>> pq;
      for (int p = st.nI; p < nc; ++p) pq.emplace(0, -nv[p], p);
      while (!pq.empty()) {
        const auto [ns, nw, p] = pq.top();
        pq.pop();
        if (st.colour[p] >= 0 || -ns != (int)seen[p].size()) continue;   // stale entry
        int c = 0;
        for (const int32_t x : seen[p]) {
          if (x == c) ++c;
          else if (x > c) break;
        }
        st.colour[p] = c;
        st.ncolours = std::max(st.ncolours, c + 1);
        for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
          const int q = st.adj[e];
          if (q < st.nI || q == p || st.colour[q] >= 0) continue;
          auto& sq = seen[q];
          const auto it = std::lower_bound(sq.begin(), sq.end(), c);
          if (it != sq.end() && *it == c) continue;
          sq.insert(it, c);
          pq.emplace(-(int)sq.size(), -nv[q], q);
        }
      }
    }
    nv_prev.swap(nv);
    st.order.clear();
    for (int p = st.nI; p < nc; ++p) st.order.push_back(p);
    std::stable_sort(st.order.begin(), st.order.end(),
                     [&](int a, int b) { return st.colour[a] < st.colour[b]; });
    st.sparsified = l >= 1 && l <= D - skip;
  }
  P.steps[0].parent.assign(P.steps[0].nc, -1);
  for (int l = 0; l <= D; ++l)
    if (P.steps[l].parent.empty()) P.steps[l].parent.assign(P.steps[l].nc, -1);
  // the lists of step l read step l - 1's structure only
  parallel_for(D + 1, host_threads(P.nnz), [&](int l) { build_numeric_lists(P, l); });
}

void merge_plans(Plan& M, const std::vector<const Plan*>& parts, int skip) {
  const int np = (int)parts.size();
  int D = 0;
  for (const Plan* q : parts) D = std::max(D, q->depth);
  M.depth = D;
  M.skip = skip;
  M.dim = parts.empty() ? 0 : parts[0]->dim;
  std::vector<int64_t> voff(np + 1, 0), eoff(np + 1, 0);
  for (int i = 0; i < np; ++i) {
    voff[i + 1] = voff[i] + parts[i]->n;
    eoff[i + 1] = eoff[i] + parts[i]->nnz;
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
    const Plan& q = *parts[i];
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
  auto own = [&](int i, int lm) { return lm - (D - parts[i]->depth); };   // problem step
  for (int lm = 0; lm <= D; ++lm) {
    StepPlan& S = M.steps[lm];
    S.l = lm;
    int nI = 0, nF = 0;
    for (int i = 0; i < np; ++i) {
      const int l = own(i, lm);
      ioff[lm][i] = nI;
      foff[lm][i] = nF;
      if (l < 0) continue;
      nI += parts[i]->steps[l].nI;
      nF += parts[i]->steps[l].nc - parts[i]->steps[l].nI;
    }
    S.nI = nI;
    S.nc = nI + nF;
    S.sparsified = lm >= 1 && lm <= D - skip;
    S.seg_ioff = ioff[lm];
    S.seg_foff = foff[lm];
  }
  M.seg_depth.resize(np);
  for (int i = 0; i < np; ++i) M.seg_depth[i] = parts[i]->depth;
  auto map = [&](int lm, int i, int c) {
    const StepPlan& q = parts[i]->steps[own(i, lm)];
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
      const StepPlan& q = parts[i]->steps[l];
      for (int c = 0; c < q.nc; ++c) {
        const int x = map(lm, i, c);
        owner[x] = {i, c};
        S.key_lvl[x] = q.key_lvl[c] + (D - parts[i]->depth);
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
      const StepPlan& q = parts[i]->steps[own(i, lm)];
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
        const StepPlan& q = parts[i]->steps[own(i, lm)];
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
        const StepPlan& q = parts[i]->steps[parts[i]->depth];
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
  P.leaf_layout = std::move(lay);
  P.leaf_dest = std::move(dest);
  if (P.seg_off.empty()) P.seg_off = {0, n};
}

std::vector<double> graph_coords(int64_t n, const int64_t* rowptr, const int32_t* colind) {
  std::vector<int32_t> queue;
  queue.reserve((size_t)n);
  auto bfs = [&](int64_t src, std::vector<int64_t>& dist) {
    dist.assign((size_t)n, n);
    queue.clear();
    dist[src] = 0;
    queue.push_back((int32_t)src);
    for (size_t h = 0; h < queue.size(); ++h) {
      const int32_t v = queue[h];
      for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int32_t u = colind[e];
        if (u < 0 || u >= n) throw Error(SPAND_E_INVALID, "column index out of range");
        if (dist[u] == n) {
          dist[u] = dist[v] + 1;
          queue.push_back(u);
        }
      }
    }
  };
  auto farthest = [&](const auto& key) {   // largest key, lowest vertex on ties
    int64_t best = 0;
    for (int64_t v = 1; v < n; ++v)
      if (key(v) > key(best)) best = v;
    return best;
  };
  std::vector<int64_t> t, d0, d1, d2;
  bfs(0, t);
  bfs(farthest([&](int64_t v) { return t[v]; }), d0);
  bfs(farthest([&](int64_t v) { return d0[v]; }), d1);
  bfs(farthest([&](int64_t v) { return std::min(d0[v], d1[v]); }), d2);
  std::vector<double> xyz((size_t)n * 3);
  for (int64_t v = 0; v < n; ++v) {
    xyz[v * 3] = (double)d0[v];
    xyz[v * 3 + 1] = (double)d1[v];
    xyz[v * 3 + 2] = (double)d2[v];
  }
  return xyz;
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
