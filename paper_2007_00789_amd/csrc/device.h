// Work descriptors shared by the host drivers and the HIP kernels, plus the
// kernel launchers.  Every launch works on a flat array of descriptors built
// by the host planner for one step of the factorization (or one phase of the
// apply), so uneven cluster sizes batch into a single launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spand {

// Element type of the row panels and of the stored factor: R = double
// (SPAND_FP64) or float (SPAND_FP32, SPAND_FP32_BF16).  Every descriptor below
// is a template on R; the launchers are instantiated for both.

// Tie band of the pivot choice of the column-pivoted QR: columns whose
// squared trailing norm is within this relative distance of the largest count
// as tied, and the tie goes to the lowest column index.  In FP32 the band is a
// few units in the last place of a float (the pivot order there is only
// required to be deterministic, not to match the FP64 oracle's).
template <class R> struct PivotTie;
template <> struct PivotTie<double> { static constexpr double rtol = 1e-8; };
template <> struct PivotTie<float> { static constexpr double rtol = 4e-7; };
constexpr double kPivotTieRtol = PivotTie<double>::rtol;

// X = L^{-1} where A = L L^T (lower triangle of A read, ld lda = n; X: n x n,
// ld n).  Blocks larger than 64 are factored in place in A, which must be
// dead after the call.
template <class R>
struct PotrfDescT {
  const R* A;
  R* X;
  int32_t lda, n;
  int32_t cluster;   // reported on breakdown
  int32_t pad;
};
using PotrfDesc = PotrfDescT<double>;

// One term of a multi-term GEMM: op(A) (m x k) times op(B) (k x n).
template <class R>
struct GemmTermT {
  const R* A;
  const R* B;
  int32_t lda, ldb, k, pad;
};

// C = beta C + alpha sum_terms op(A) op(B); when C2 != nullptr the result is
// also stored transposed into C2 (ld ldc2).  lower_only: only tiles that touch
// the lower triangle (square C) are computed.
template <class R>
struct GemmDescT {
  R* C;
  R* C2;
  int64_t term0, term1;
  int32_t ldc, ldc2, m, n;
  int32_t transA, transB, lower_only, pad;
  double alpha, beta;
};

struct TileRef {
  int32_t desc, ti, tj, pad;
};

// Arithmetic of a GEMM launch: the panels' own precision (FP64 on the FP64
// matrix cores, FP32 on the FP32 matrix cores), or (R = float only) the BF16
// matrix cores: each FP32 operand split into two BF16 terms, three BF16
// products per operand pair, accumulated in FP32.
enum GemmMode { kGemmNative = 0, kGemmBf16 = 1 };

// Early-stopping column-pivoted QR of one interface (Alg. 1).
template <class R>
struct CpqrNbrT {
  R* blk_wp;         // block (w, p) in w's row panel (transposed write-back)
  int64_t col;       // column offset of block (p, w) in p's row panel
  int32_t w, ldw;
};
template <class R>
struct CpqrDescT {
  R* panel;          // p's row panel, ld = a
  R* Y;              // a x kmax workspace; holds Q^T W afterwards (E lives in rows r..)
  R* V;              // a x min(a, kmax) Householder vectors (unit diagonal stored)
  R* tau;            // min(a, kmax)
  R* T;              // nref x nref (ld nref) triangular factor of the WY form
  int64_t nb0, nb1;  // neighbour range
  int64_t diag_col;  // column offset of the diagonal block (p, p)
  int32_t a, kmax, p, pad;
};

// One interface of a cooperative QR launch: G workgroups share the columns of
// W, at most ncap each.  The launcher plans all G workgroups of a group on one
// XCD (planned block index = xcd + 8 * slot) so that the group synchronizes
// through that XCD's L2; each workgroup takes the next planned index of the
// XCD it runs on, and the kernel verifies the placement (xcd < 0: treat as
// not placed; a misplaced group leaves with bit 2 of the error flag set).
template <class R>
struct CoopDescT {
  CpqrDescT<R> d;
  int32_t* sync;     // kCoopSyncInts ints, zeroed by the launcher: [0] placement
                     // check counter, barrier flags from [kCoopFlag64] (64-bit,
                     // two parities)
  double* xch;       // exchange buffer, coop_xch_doubles(G, a)
  int32_t G, xcd, ncap, list_cap;  // list_cap <= 32 tie candidates per workgroup
  int32_t ncap_lds;  // columns per workgroup held in LDS; the rest of its
                     // columns (up to ncap) stay in the panel (global memory)
  int32_t pad;
};
constexpr int kCoopMaxGroup = 32;
constexpr int kCoopList = 32;           // tie candidates exchanged per workgroup
constexpr int kCoopXcds = 8;             // XCDs of an MI355X; block b runs on XCD b % 8
constexpr size_t kCoopLdsBytes = 140 * 1024;
inline int64_t coop_xch_doubles(int G, int a) {
  return 2 * (int64_t)G * (2 + 2 * kCoopList) + (int64_t)(2 * G + 1) * (a + 1) + G;
}
// dynamic LDS of the LDS-resident cooperative QR: the slice (a x ncap), its
// norms and the Householder vector (elements of R), and the addresses of the
// columns kept in the panel
template <class R>
__host__ __device__ inline size_t coop_lds_ptr_offset(int a, int ncap, int ncap_lds) {
  return (((size_t)a * ncap_lds + ncap + a) * sizeof(R) + 7) / 8 * 8;
}
template <class R>
inline size_t coop_lds_bytes(int a, int ncap, int ncap_lds) {
  return coop_lds_ptr_offset<R>(a, ncap, ncap_lds) + (size_t)(ncap - ncap_lds) * sizeof(R*);
}
// columns of an a-row slice that fit the cooperative QR's LDS
template <class R>
inline int64_t coop_cols(int a) {
  return ((int64_t)(kCoopLdsBytes / sizeof(R)) - a) / (a + 1);
}
// a workgroup may hold up to this many times its LDS columns, the rest in the
// panel, when an interface is too wide for kCoopMaxGroup workgroups' LDS
constexpr int kCoopOverflow = 4;
constexpr int kCoopSyncInts = 192;       // 768 bytes per group
constexpr int kCoopFlag64 = 64;          // 2 x kCoopMaxGroup 64-bit flags (LDS-resident QR)

// Triangular factor of the compact WY form of one interface's n reflectors
// (V a x n, T n x n, both column-major); T holds V^T V in its lower triangle
// on entry.
template <class R>
struct WyDescT {
  const R* V;
  const R* tau;
  R* T;
  R* X;              // n > kWyLdsN: n x n scratch for the blocked inverse
  int32_t a, n;
};
constexpr int kWyThreads = 1024;
constexpr int kWyLdsN = 143;   // 143^2 doubles fit in the 160 KiB of LDS

// Dense block copy (merge of children's blocks into parent panels), with a
// conversion when the element types differ.
template <class S, class D>
struct CopyDescT {
  const S* src;
  D* dst;
  int32_t lds, ldd, m, n;
};

template <class R>
void launch_fill(R* p, int64_t n, double v, hipStream_t s);
template <class R>
void launch_scatter(const double* vals, const int64_t* dest, int64_t nnz, R* panels, hipStream_t s);
// X = L^{-1} with A = L L^T for count blocks of at most max_n rows (info[i]:
// 0, or the 1-based column of the first non-positive pivot of block i, whose
// X is then left zero).  launch_potrf_inv: max_n <= 64 runs one wave per
// block, larger max_n one workgroup per block; launch_potrf_blocks always
// runs one workgroup per block (256 threads when max_n <= 64, else 16 waves
// with the tile products on the FP64 matrix cores).  Blocks above 64 rows are
// factored in place: their diagonal block in A (ld n) is overwritten.  Blocks
// above 64 rows exist in FP64 only (the FP32 forms factor them in FP64).
template <class R>
void launch_potrf_inv(const PotrfDescT<R>* d, int32_t count, int32_t max_n, int32_t* info,
                      hipStream_t s);
template <class R>
void launch_potrf_blocks(const PotrfDescT<R>* d, int32_t count, int32_t max_n, int32_t* info,
                         hipStream_t s);
// tile: the output tile of the launch's TileRefs, kGemmTile (64) or kGemmTileL
// (128: four 64 x 64 wave quadrants, double-buffered k-slabs)
template <class R>
void launch_gemm(const GemmDescT<R>* d, const GemmTermT<R>* t, const TileRef* tiles, int64_t ntiles,
                 GemmMode mode, int tile, hipStream_t s);
// blocks of at most kGemmSmallN x kGemmSmallN (FP64 or FP32 arithmetic): one
// wave per block; refs[i].desc names the descriptor of the i-th block
constexpr int kGemmSmallN = 32;
template <class R>
void launch_gemm_small(const GemmDescT<R>* d, const GemmTermT<R>* t, const TileRef* refs,
                       int64_t count, hipStream_t s);
template <class R>
void launch_cpqr(const CpqrDescT<R>* d, const CpqrNbrT<R>* nb, int32_t count, int32_t* n_cur,
                 int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps, double eps_stop,
                 int32_t max_a, int32_t max_k, hipStream_t s);
template <class S, class D>
void launch_copy(const CopyDescT<S, D>* d, int64_t count, hipStream_t s);
template <class R>
void launch_wy_t(const WyDescT<R>* d, int32_t count, hipStream_t s);
// maximum co-resident workgroups of the cooperative QR for a given LDS size
// (panel: the instance that supports columns kept in the row panel)
template <class R>
int coop_max_blocks(size_t lds_bytes, bool panel);
void launch_fill_int(int32_t* p, int64_t n, hipStream_t s);
// Group memberships are codes group * kCoopMaxGroup + member, or -1 (idle),
// for the nblocks planned blocks b = xcd + 8 * slot.  The grid has ngrid
// workgroups (a multiple of 8 that fills every compute unit, so that every
// XCD holds ngrid / 8 of them); at entry a workgroup takes the next slot of its
// XCD from the 8 counters at xcd_slot (zero on entry: the caller clears them)
// and runs the planned block of that index, if any.  blk_ptr == nullptr: block b holds the
// one membership blk_map[b].  Otherwise block b runs the memberships
// blk_map[blk_ptr[b] .. blk_ptr[b + 1]) one after the other.  The caller numbers the groups in rounds (the groups of a round
// fit the co-resident blocks together) and lists every block's memberships in
// round order, so that a group waits only for groups of earlier rounds, which
// all complete.  The launch first clears the nsync barrier words at `sync`
// (each group's CoopDesc::sync points into them); nsync = 0 when the caller
// has cleared them already.
template <class R>
hipError_t launch_cpqr_coop(const CoopDescT<R>* d, const CpqrNbrT<R>* nb, const int32_t* blk_map,
                            const int32_t* blk_ptr, int32_t nblocks, int32_t ngrid,
                            int32_t* xcd_slot, int32_t* sync, int32_t nsync, int32_t* n_cur,
                            int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps,
                            double eps_stop, int32_t* err, size_t lds_bytes, bool panel,
                            hipStream_t s);

constexpr int kGemmTile = 64;
constexpr int kGemmTileL = 128;
constexpr int kCpqrMaxK = 12288;      // trailing norms of a CPQR live in LDS

}  // namespace spand
