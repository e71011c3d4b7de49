// Internal structures of libspand (host side).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/spand.h"

namespace spand {

// Error carried from deep inside the library to the C ABI boundary.
struct Error : std::runtime_error {
  spand_status code;
  Error(spand_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SPAND_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::spand::Error(e_ == hipErrorOutOfMemory ? SPAND_E_OOM : SPAND_E_HIP,         \
                           std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

// ---------------------------------------------------------------------------
// Symbolic plan (result of analyze)
// ---------------------------------------------------------------------------
struct StepPlan {
  int l = 0;
  int nI = 0;                          // interiors are clusters [0, nI)
  int nc = 0;                          // clusters [nI, nc) are interfaces
  bool sparsified = false;
  std::vector<int64_t> key_lvl, key_prefix;
  std::vector<int64_t> adj_ptr;        // CSR of the cluster adjacency (sorted, incl. self)
  std::vector<int32_t> adj;
  std::vector<int32_t> colour;         // -1 for interiors
  int ncolours = 0;
  std::vector<int32_t> order;          // interfaces in (colour, index) order
  std::vector<int64_t> child_ptr;      // l < depth: children in step l+1
  std::vector<int32_t> child;
  std::vector<int32_t> parent;         // index in step l-1 (-1 for interiors / l == 0)
  std::vector<int64_t> vert_ptr;       // l == depth: vertices of each cluster, ascending
  std::vector<int32_t> verts;
  // Structural lists for the numeric factorization (they depend on the
  // pattern only; sizes and addresses are filled in per factorization).
  std::vector<int64_t> adj_rev;        // entry e = (c, w): position of c in w's list
  // Schur update of one block B_{w1 w2} (w1 <= w2 interfaces sharing an
  // interior): e = position of w2 in w1's list; its terms [t0, t1) in
  // ascending interior order give s and the positions of w1 and w2 in s's list
  struct SchurTarget {
    int32_t w1, w2;
    int64_t e, t0, t1;
  };
  struct SchurTerm {
    int32_t s, pad;
    int64_t e1, e2;
  };
  std::vector<SchurTarget> schur;
  std::vector<SchurTerm> schur_terms;
  // merge of this step into step l-1: child block (ci, cj) (cj at position ee
  // of ci's list) goes to parent block (P, Q = adj[e]) of step l-1
  struct MergeCopy {
    int32_t P, ci, cj, pad;
    int64_t e, ee;
  };
  std::vector<MergeCopy> merge;
  // batch plans: per problem, the offsets of its interiors among the step's
  // interiors and of its interfaces among the step's interfaces (problems not
  // present at this step keep the running offset)
  std::vector<int32_t> seg_ioff, seg_foff;
};

struct PanelLayout {
  std::vector<int32_t> n;
  std::vector<int64_t> off;
  std::vector<int64_t> width;
  std::vector<int64_t> coff;   // per adjacency entry
  int64_t total = 0;
};

struct Plan {
  int64_t n = 0, nnz = 0;
  int depth = 0, skip = 4, dim = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<int32_t> lvl;
  std::vector<int64_t> path;
  std::vector<int64_t> perm;
  std::vector<StepPlan> steps;         // indexed by l
  // device copies of the pattern (SpMV) and of the leaf assembly map
  int device = 0;
  int64_t* d_rowptr = nullptr;
  int32_t* d_colind = nullptr;
  int64_t* d_leaf_dest = nullptr;      // nnz: destination of each value in the leaf panels
  std::vector<int64_t> leaf_dest;      // host copy of the same map
  int64_t leaf_panel_elems = 0;
  std::vector<int64_t> leaf_panel_off; // per leaf-step cluster
  PanelLayout leaf_layout;             // panel layout of the leaf step
  // independent problems of a batch plan: problem s owns rows seg_off[s] ..
  // seg_off[s+1]-1 (one segment for a single problem)
  std::vector<int64_t> seg_off;
  std::vector<int32_t> seg_id;         // segment of every row (batch plans only)
  std::vector<int32_t> seg_depth;      // batch plans: each problem's own depth
  int32_t* d_seg_id = nullptr;
  int64_t* d_seg_off = nullptr;
  ~Plan();
};

void analyze_plan(Plan& P, const int64_t* rowptr, const int32_t* colind, const double* coords,
                  int dim, int depth, int skip);
// One plan for independent problems (a block-diagonal system): problem i's
// rows follow those of problems < i, and its own step l becomes step
// l + (D - D_i) with D the largest depth, so every problem keeps its own
// levels, and the rule 1 <= l <= D_i - skip for sparsified steps becomes
// 1 <= l' <= D - skip for all of them.
void merge_plans(Plan& M, const std::vector<const Plan*>& parts, int skip);
// destination of every CSR value in the leaf-step row panels
void build_leaf_map(Plan& P);
// Coordinates for a matrix given without any (coordinate-free analysis): for
// every vertex, its hop distances in the graph of A to three landmarks picked
// by farthest-point sampling: l0 the vertex farthest from vertex 0, l1 the
// vertex farthest from l0, l2 the vertex whose distance to the nearer of l0
// and l1 is largest (ties: lowest vertex id; unreachable vertices at distance
// n).  Integer work, so the coordinate bisection on them is exact.  n x 3,
// row-major.
std::vector<double> graph_coords(int64_t n, const int64_t* rowptr, const int32_t* colind);

// Layout of one step's row panels: cluster c holds rows n[c] x width[c] in
// column-major order (ld = n[c]) at offset off[c]; the block (c, adj[e]) starts
// at column coff[e].
PanelLayout make_layout(const StepPlan& st, const std::vector<int32_t>& sizes);

}  // namespace spand
