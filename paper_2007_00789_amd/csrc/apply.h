// Descriptors of the preconditioner apply and the PCG building blocks.
//
// The vector z (n x nrhs, column-major, ld n) is indexed by original vertex
// numbers; a cluster's current variables are a list of positions into it.
// Forward (z <- L^{-1} z), per step l = depth ... 0:
//   ApInt  (one workgroup per interior):  z_s <- L_s^{-1} z_s,
//          t_s = G_s^T z_s written to a scratch buffer;
//   ApGat  (one workgroup per interface): z_w -= sum_s t_s[w] (ascending s),
//          then z_w <- Z_w^{-1} z_w on sparsified steps;
//   per colour: ApSp  z_p <- Q_p^T z_p; ApEt tiles t_p = E_p^T z_f (second order);
//               ApGat z_w -= sum_p t_p[w] (ascending p).
// Backward (y <- L^{-T} y) runs the transposes in reverse.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spand {

// Factor entries (L^{-1}, G, Z^{-1}, V, T, V T, E, M) are of the factor's
// element type (double, or float in the FP32 forms; the launchers take it as
// `f32`); vectors and scratch are always double.
struct ApInt {
  const void* Linv;        // n x n
  const void* G;           // n x k (G_s = L_s^{-1} B_sW)
  const int32_t* pos;      // n
  const int32_t* nbr_pos;  // k
  int64_t toff;            // scratch offset (units of one right-hand side)
  int32_t n, k;
};

// Split GEMV over many workgroups, for the large interiors of the top levels
// (one workgroup per interior leaves most of the chip idle there).  A
// descriptor is one matrix product with its operand and result addresses:
//  rows kernel (tasks of kApMvRB rows): out_i = base_i - sum_j M[i, j] x_j
//    (base from z at bpos; without bpos, out_i = + sum_j M[i, j] x_j)
//  cols kernel (tasks of 4 x kApMvCB columns): out_c = sum_i M[i, c] x_i;
//    the task of column 0 also writes x_i to z at wpos when wpos is set.
// x_j: z[xpos[j] + r ldz] if xpos, else S[xoff nrhs + j + r xld];
// out: z[opos[i] + r ldz] if opos, else O[ooff nrhs + i + r old]
// (scratch offsets in units of one right-hand side, as the T scratch).
// tri = 1: M is lower triangular (zeros above the diagonal are skipped).
struct ApMv {
  const void* M;
  const int32_t* xpos;
  const int32_t* opos;
  const int32_t* bpos;
  const int32_t* wpos;
  int64_t ld, xoff, xld, ooff, old;
  int32_t rows, cols, tri, pad;
};
struct ApMvTask {
  int32_t mv;   // descriptor
  int32_t i0;   // first row (rows kernel) or column (cols kernel)
};
constexpr int kApMvRB = 16;
constexpr int kApMvCB = 8;
// interiors per step below which the split kernels are used
constexpr int kApSplitBelow = 512;

struct ApSrc {             // one slice of a scratch vector subtracted from a target
  int64_t toff;            // scratch offset of the producer (units of one rhs)
  int32_t col, ld;         // slice start inside the producer's vector, producer length
};

struct ApGat {
  const int32_t* pos;      // target positions (first n)
  const void* Zinv;        // nullable: scale after the subtraction (forward only)
  int64_t src0, src1;      // range in the ApSrc list
  int64_t yoff;            // split scaling: the difference goes to the scratch at yoff
  int32_t n, split;        // split = 1: no scaling here (a split GEMV applies Zinv)
};

struct ApSp {
  const void* V;           // a x nref reflectors (ld a, zero above the unit diagonal)
  const void* tau;         // nref
  const void* T;           // nref x nref: Q = I - V T V^T
  const void* VT;          // a x nref (ld a): V T
  const void* Et;          // E^T: k x (f1-f0), column i = row f0+i of Q^T W (ld lde); nullable
  const int32_t* pos;      // a
  const int32_t* nbr_pos;  // k
  int64_t toff;
  int64_t lde;
  int64_t part0;           // backward: first partial-sum slot of the E tiles (units of one rhs)
  int64_t uoff;            // offset of u = (VT)^T x or V^T y in the colour's scratch
  int32_t a, nref, f0, f1, k, ntiles;
};

// The wide WY apply of one colour runs as two launches spread over blocks of
// every interface: dots (u = M^T x over kApWyCB columns of M per task) and
// update (x -= N u over kApWyRB rows per task), with (M, N) = (VT, V) forward
// (x <- Q^T x) and (V, VT) backward (y <- Q y, after the E-tile partial sums
// are subtracted from the fine rows).
struct ApWyTask {
  int32_t sp;   // descriptor of the interface
  int32_t i0;   // first column (dots) or row (update)
};
constexpr int kApWyThreads = 256;
constexpr int kApWyCB = 8;
constexpr int kApWyRB = 16;

// One tile of at most kEtTileF (forward) or kEtTileB (backward) columns of an interface's E (second order:
// E = rows f0.. of Q^T W, stored transposed, element (c, i) = E[i, c] at
// Et[c + i*lde]).  Forward: t[c0 + c] = sum_i E[i, c0 + c] z_f[i] for the
// tile's columns, into the interface's scratch vector (offset off, length k).
// Backward: part[i] = sum_c E[i, c0 + c] y_W[c0 + c] for every fine row i, into
// the tile's partial-sum slot (offset off, length nf).
struct ApEt {
  const void* Et;
  const int32_t* pos;      // forward: positions of the nf fine rows; backward: of the k columns
  int64_t lde;
  int64_t off;             // units of one right-hand side
  int32_t nf, k, c0, cn;
};
constexpr int kEtTileF = 64;    // columns per forward E tile
constexpr int kEtTileB = 256;   // columns per backward E tile

struct ApScale {
  const void* Zinv;
  const int32_t* pos;
  int32_t n, pad;
};

// f32: the factor entries of the descriptors are floats (else doubles)
void launch_ap_int_fwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       double* T, int32_t max_n, bool f32, hipStream_t s);
// Y: scratch of the split scaling (descriptors with split = 1), else unused
void launch_ap_gather(const ApGat* d, const ApSrc* src, int32_t count, double* z, int64_t ldz,
                      int32_t nrhs, const double* T, int32_t max_n, bool f32, hipStream_t s,
                      double* Y = nullptr);
// split GEMV kernels (S: operand scratch, O: result scratch)
void launch_ap_mv_rows(const ApMvTask* t, int32_t count, const ApMv* d, double* z, int64_t ldz,
                       int32_t nrhs, const double* S, double* O, bool f32, hipStream_t s);
void launch_ap_mv_cols(const ApMvTask* t, int32_t count, const ApMv* d, double* z, int64_t ldz,
                       int32_t nrhs, const double* S, double* O, bool f32, hipStream_t s);
// wide WY apply, dots then update (fwd = 1: Q^T; 0: Q, after the partial
// sums P); U: the colour's u vectors, usz doubles per right-hand side
void launch_ap_wy_dots(const ApWyTask* t, int32_t count, const ApSp* d, const double* z,
                       int64_t ldz, int32_t nrhs, const double* P, double* U, int64_t usz, int fwd,
                       bool f32, hipStream_t s);
void launch_ap_wy_update(const ApWyTask* t, int32_t count, const ApSp* d, double* z, int64_t ldz,
                         int32_t nrhs, const double* P, const double* U, int64_t usz, int fwd,
                         bool f32, hipStream_t s);
// E tiles, forward (t = E^T z_f) or backward (partial sums of E y_W)
void launch_ap_et_fwd(const ApEt* d, int32_t count, const double* z, int64_t ldz, int32_t nrhs,
                      double* T, int32_t max_nf, bool f32, hipStream_t s);
void launch_ap_et_bwd(const ApEt* d, int32_t count, const double* z, int64_t ldz, int32_t nrhs,
                      double* P, bool f32, hipStream_t s);
void launch_ap_scale_bwd(const ApScale* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                         int32_t max_n, bool f32, hipStream_t s);
void launch_ap_int_bwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       int32_t max_n, bool f32, hipStream_t s);

// PCG helpers.  Vectors are n x nrhs (ld n); the rows are split into nseg
// segments (independent problems of a batch, seg_off: nseg + 1 offsets on the
// device, seg_id: the segment of every row, nullptr when nseg == 1), and every
// scalar is per (segment s, column c), stored at s * nrhs + c.
void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                 int32_t nrhs, const double* x, double* y, hipStream_t s);
// out[s, c] = sum_{i in s} x[i,c] * y[i,c] (deterministic two-stage reduction)
void launch_dot(const double* x, const double* y, int64_t n, int32_t nrhs, const int64_t* seg_off,
                int32_t nseg, double* partial, double* out, hipStream_t s);
// alpha = rho/pq for active (s, c); x += alpha p; r -= alpha q
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rho,
                   const double* pq, const int32_t* active, const int32_t* seg_id, int64_t n,
                   int32_t nrhs, hipStream_t s);
// p = z + (rho_new/rho) p for active (s, c) (p = z when first != 0); rho <- rho_new
void launch_pcg_p(double* p, const double* z, double* rho, const double* rho_new,
                  const int32_t* active, const int32_t* seg_id, int64_t n, int32_t nrhs,
                  int32_t nseg, int32_t first, hipStream_t s);
// y = b - y
void launch_residual(const double* b, double* y, int64_t n, int32_t nrhs, hipStream_t s);
void launch_copy_vec(const double* src, double* dst, int64_t count, hipStream_t s);
// prescale: d = diag(A)^{-1/2} (*bad: lowest row with a non-positive or missing
// diagonal, INT32_MAX if none) and out = D^{-1/2} A D^{-1/2} in A's CSR order
void launch_prescale(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                     double* d, double* out, int32_t* bad, hipStream_t s);
// y = d o x, column by column (x and y may alias)
void launch_scale_vec(const double* x, const double* d, double* y, int64_t n, int32_t nrhs,
                      hipStream_t s);
// blocks per (segment, column) of launch_dot and the size of its partial buffer
int32_t dot_blocks(int32_t nseg);

constexpr int kDotBlocks = 256;

}  // namespace spand
