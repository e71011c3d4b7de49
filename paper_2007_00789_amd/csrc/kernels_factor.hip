// HIP kernels of the factorization (gfx950).  Every kernel is a template on
// the element type R of the row panels and of the stored factor (double for
// SPAND_FP64, float for the FP32 forms), except the large-block Cholesky,
// which exists in FP64 only.
//
//  k_potrf_inv_small : batched Cholesky + triangular inverse of blocks of at
//                most 64 rows, one wave per block, the block in registers.
//  k_potrf_inv : the same, one workgroup per block, in LDS.
//  k_potrf_inv_big : blocks larger than 64 rows, 16 waves per block: 64x64
//                diagonal tiles in LDS, the tile products on the FP64 matrix
//                cores, factored in place in global memory.
//  k_gemm      : batched multi-term GEMM over 64x64 output tiles; serves the
//                TRSM of the interiors (as a product with L^{-1}), the Schur
//                complement scatter (one tile list per target block, terms in
//                ascending interior order, so the sums are deterministic and
//                atomic-free), and the two-sided interface scaling.
//  k_cpqr      : early-stopping column-pivoted Householder QR of one
//                interface per workgroup (Alg. 1), with exact recomputation of
//                every trailing column norm fused into the reflector update.
//  k_fill, k_scatter, k_copy : assembly of the leaf panels from CSR values and
//                the merge of child blocks into parent panels.
#include <climits>
#include <type_traits>

#include "device.h"

namespace spand {

namespace {

constexpr int kWave = 64;

// DPP move of a double (two 32-bit halves); lanes whose source is invalid read 0.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// DPP move of a float.
template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}

// Sum over the 64 lanes, returned to every lane.  Quad permutations and row
// rotations reduce each row of 16 lanes; row broadcasts 15 and 31 then carry
// the row sums upward so that lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  v += dpp_move<0x142>(v);  // row_bcast:15
  v += dpp_move<0x143>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
// Sum over each group of 8 lanes, returned to all 8: two quad permutations and
// a half-row mirror.
template <class R>
__device__ __forceinline__ R group8_sum(R v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  return v;
}
template <class R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

// Block-wide reductions through a small LDS scratch (one slot per wave).  All
// threads receive the result.  The scratch is reused, so each call ends with a
// barrier.
template <int NT>
__device__ double block_sum(double v, double* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];  // same order in every thread
  __syncthreads();
  return s;
}
template <int NT>
__device__ double block_max(double v, double* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}
template <int NT>
__device__ int block_min_int(int v, int* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  v = wave_min_int(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  int s = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s = min(s, red[w]);
  __syncthreads();
  return s;
}

// 1/sqrt(v) for a positive normal v: the hardware estimate refined by two
// Newton steps y <- y (3 - v y^2) / 2, which leaves a few units in the last
// place.  The pivots need no correctly rounded root, and this is a short
// dependent chain where sqrt and two divisions are a long one.
__device__ __forceinline__ double rsqrt_nr(double v) {
  double y = __builtin_amdgcn_rsq(v);
  const double h = 0.5 * v;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
// FP32: the hardware estimate and one Newton step.
__device__ __forceinline__ float rsqrt_nr(float v) {
  float y = __builtin_amdgcn_rsqf(v);
  const float h = 0.5f * v;
  return y * fmaf(-h * y, y, 1.5f);
}

// ---------------------------------------------------------------------------
// Cholesky of an n x n SPD block (n <= 64, column-major in LDS, lower triangle
// read).  Right-looking with one barrier per column: every thread reads the
// pivot v, updates its share of the trailing lower triangle with the unscaled
// column (S_ic -= S_ij S_cj / v), and scales the previous column, which is no
// longer read.  Returns 0 or the 1-based column of the first non-positive pivot.
// ---------------------------------------------------------------------------
template <int NT, class R>
__device__ int chol_inplace(R* S, int n, int ld) {
  constexpr int TX = 16, TY = NT / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  R vprev = 0, rprev = 0;
  for (int j = 0; j <= n; ++j) {
    if (j > 0) {   // finish column j-1: l_jj = v rsqrt(v), l_ij = s_ij rsqrt(v)
      const int jp = j - 1;
      for (int i = j + threadIdx.x; i < n; i += NT) S[i + (int64_t)jp * ld] *= rprev;
      if (threadIdx.x == 0) S[jp + (int64_t)jp * ld] = vprev * rprev;
    }
    if (j == n) break;
    const R v = S[j + (int64_t)j * ld];
    if (!(v > R(0))) return j + 1;   // every thread reads the same value
    const R rs = rsqrt_nr(v), rv = rs * rs;
    for (int c = j + 1 + ty; c < n; c += TY) {
      const R scj = S[c + (int64_t)j * ld] * rv;
      for (int i = c + tx; i < n; i += TX)
        S[i + (int64_t)c * ld] = fma(-S[i + (int64_t)j * ld], scj, S[i + (int64_t)c * ld]);
    }
    __syncthreads();
    vprev = v;
    rprev = rs;
  }
  __syncthreads();
  return 0;
}

// X = L^{-1} for a lower triangular n x n L (n <= 64, in LDS, X not aliasing
// L; X is zeroed above the diagonal).  16 x 16 blocks: wave I inverts diagonal
// block I by forward substitution (lane c builds column c), then the blocks
// below the diagonal follow one block diagonal at a time,
// X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ.  tmp: 768 doubles of LDS (first the
// reciprocals of L's diagonal).
template <int NT, class R>
__device__ void trinv(const R* L, int ldl, R* X, int ldx, int n, R* tmp) {
  static_assert(NT >= 256, "one wave per 16-row diagonal block");
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int nbk = (n + 15) / 16;
  for (int c = wid; c < n; c += NT / kWave)
    for (int i = lane; i < n; i += kWave) X[i + (int64_t)c * ldx] = 0;
  for (int i = tid; i < n; i += NT) tmp[i] = R(1) / L[i + (int64_t)i * ldl];
  __syncthreads();
  if (wid < nbk && lane < 16) {
    const int b0 = wid * 16, bw = min(16, n - b0), c = lane;
    if (c < bw) {
      const int gc = b0 + c;
      X[gc + (int64_t)gc * ldx] = tmp[gc];
      for (int i = c + 1; i < bw; ++i) {
        const int gi = b0 + i;
        R acc = 0;
        for (int k = c; k < i; ++k)
          acc = fma(L[gi + (int64_t)(b0 + k) * ldl], X[b0 + k + (int64_t)gc * ldx], acc);
        X[gi + (int64_t)gc * ldx] = -acc * tmp[gi];
      }
    }
  }
  __syncthreads();
  for (int dd = 1; dd < nbk; ++dd) {
    const int nblk = nbk - dd;
    for (int idx = tid; idx < nblk * 256; idx += NT) {   // S_IJ = sum_K L_IK X_KJ
      const int q = idx >> 8, e = idx & 255, ii = e & 15, jj = e >> 4;
      const int I = q + dd, i = I * 16 + ii, j = q * 16 + jj;
      R acc = 0;
      if (i < n && j < n)
        for (int k = q * 16; k < I * 16; ++k)
          acc = fma(L[i + (int64_t)k * ldl], X[k + (int64_t)j * ldx], acc);
      tmp[idx] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < nblk * 256; idx += NT) {   // X_IJ = -X_II S_IJ
      const int q = idx >> 8, e = idx & 255, ii = e & 15, jj = e >> 4;
      const int I = q + dd, i = I * 16 + ii, j = q * 16 + jj;
      if (i < n && j < n) {
        R acc = 0;
        for (int k = I * 16; k <= i; ++k)
          acc = fma(X[i + (int64_t)k * ldx], tmp[(q << 8) + (k - I * 16) + jj * 16], acc);
        X[i + (int64_t)j * ldx] = -acc;
      }
    }
    __syncthreads();
  }
}

constexpr int kPotrfThreads = 256;
constexpr int kNb = 64;          // tile of the blocked Cholesky / inverse
constexpr int kTl = kNb + 1;     // padded leading dimension of LDS tiles

// LDS tile <- rows x cols block of a column-major global matrix (zero padded).
template <class R>
__device__ __forceinline__ void tile_load(R* t, const R* g, int64_t ld, int rows, int cols) {
  for (int idx = threadIdx.x; idx < kNb * kNb; idx += kPotrfThreads) {
    const int i = idx % kNb, j = idx / kNb;
    t[i + j * kTl] = (i < rows && j < cols) ? g[i + j * ld] : R(0);
  }
}

// acc (4x4 per thread, rows tx+16r, cols ty+16c) += A * op(B) over kk < kdim,
// A and B 64x64 LDS tiles; transB: B is used transposed.
template <class R>
__device__ __forceinline__ void tile_mma(R (&acc)[4][4], const R* A, const R* B, int kdim,
                                         bool transB) {
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  for (int kk = 0; kk < kdim; ++kk) {
    R a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = A[tx + 16 * r + kk * kTl];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = transB ? B[ty + 16 * c + kk * kTl] : B[kk + (ty + 16 * c) * kTl];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
  }
}

template <class R>
__device__ __forceinline__ void acc_zero(R (&acc)[4][4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0;
}

// Off-diagonal tiles of X = L^{-1} for a lower triangular L (in A, ld n) whose
// diagonal tiles of X are already in place, column block by column block:
// X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ.  The strictly upper part of X is
// zeroed.  LDS: two 64x65 tiles.
template <class R>
__device__ void lower_inv_offdiag(const R* A, R* X, int n, R* lds) {
  R* T1 = lds + kNb * kTl;
  R* T2 = lds + 2 * kNb * kTl;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int nb = (n + kNb - 1) / kNb;
  R acc[4][4];
  // off-diagonal tiles of X = L^{-1}, column block by column block
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = jb * kNb, jw = min(kNb, n - j0);
    for (int ib = jb + 1; ib < nb; ++ib) {
      const int i0 = ib * kNb, iw = min(kNb, n - i0);
      acc_zero(acc);
      for (int kb = jb; kb < ib; ++kb) {
        const int k0 = kb * kNb, kw = min(kNb, n - k0);
        tile_load(T1, A + i0 + (int64_t)k0 * n, n, iw, kw);   // L_IK
        tile_load(T2, X + k0 + (int64_t)j0 * n, n, kw, jw);   // X_KJ
        __syncthreads();
        tile_mma(acc, T1, T2, kw, false);
        __syncthreads();
      }
      // T1 <- S = sum, then X_IJ = -X_II S
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) T1[tx + 16 * r + (ty + 16 * c) * kTl] = acc[r][c];
      tile_load(T2, X + i0 + (int64_t)i0 * n, n, iw, iw);
      __syncthreads();
      acc_zero(acc);
      tile_mma(acc, T2, T1, iw, false);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int i = tx + 16 * r, j = ty + 16 * c;
          if (i < iw && j < jw) {
            X[i0 + i + (int64_t)(j0 + j) * n] = -acc[r][c];
            X[j0 + j + (int64_t)(i0 + i) * n] = 0;   // strictly upper part
          }
        }
      __syncthreads();
    }
  }
}

// Blocks of at most 64 rows, one workgroup per block, in LDS.
template <class R>
__global__ __launch_bounds__(kPotrfThreads) void k_potrf_inv(const PotrfDescT<R>* descs,
                                                             int32_t* info) {
  extern __shared__ __align__(16) char smraw[];
  R* sm = reinterpret_cast<R*>(smraw);
  const PotrfDescT<R> d = descs[blockIdx.x];
  const int n = d.n;
  if (n == 0) return;
  const int tid = threadIdx.x;
  R* S = sm;
  R* X = sm + n * n;
  R* tmp = X + n * n;
  for (int idx = tid; idx < n * n; idx += kPotrfThreads) {
    const int i = idx % n, j = idx / n;
    S[idx] = i >= j ? d.A[i + (int64_t)j * d.lda] : R(0);
  }
  __syncthreads();
  const int f = chol_inplace<kPotrfThreads>(S, n, n);
  if (f) {
    // breakdown: report it and leave a zero inverse, so that the products
    // formed with it before the flag is read stay finite
    if (tid == 0) info[blockIdx.x] = f;
    for (int idx = tid; idx < n * n; idx += kPotrfThreads) d.X[idx] = 0;
    return;
  }
  trinv<kPotrfThreads>(S, n, X, n, n, tmp);
  for (int idx = tid; idx < n * n; idx += kPotrfThreads) d.X[idx] = X[idx];
}

// ---------------------------------------------------------------------------
// Cholesky + inverse of blocks larger than one tile, 16 waves per block:
// right-looking blocked Cholesky in place, with the tile products on the FP64
// matrix cores (16 x 16 x 4 per instruction) and their operands read straight
// from global memory (the block stays in L2): the 64 x 64 diagonal tiles are
// factored and inverted in LDS, the panel below each one is
// multiplied by the tile's inverse (transposed) one 16-row strip per wave, the
// trailing lower triangle is updated by 16 x 16 subtiles spread over the
// waves, and the off-diagonal tiles of X = L^{-1} follow by tile anti-diagonals
// (X_IJ for I - J = d needs only X_KJ with K - J < d), first
// S_IJ = sum_{K=J}^{I-1} L_IK X_KJ, kept transposed in the dead upper triangle
// of A, then X_IJ = -X_II S_IJ.
// ---------------------------------------------------------------------------
constexpr int kBigThreads = 1024;
constexpr int kBigWaves = kBigThreads / kWave;

typedef double d4_t __attribute__((ext_vector_type(4)));

// Operand of one 16 x 16 x 4 step: lane l supplies row l % 16 of the 16 x 4
// left factor at column l / 16, and column l % 16 of the 4 x 16 right factor at
// row l / 16.  The 16 x 16 accumulator gives lane l rows l / 16 + 4 v,
// v = 0..3, of column l % 16 (checked on gfx950).
__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += P Q for one 16 x 16 subtile, with P(i, k) = p[i * pi + k * pk]
// (i < pm) and Q(k, j) = q[k * qk + j * qj] (j < qn), k < kdim; rows and
// columns outside the bounds read as zero.  Loads of 32 values of k are issued
// together before their 8 products.
__device__ __forceinline__ void sub_mma(d4_t& acc, const double* p, int64_t pi, int64_t pk,
                                        int pm, const double* q, int64_t qk, int64_t qj, int qn,
                                        int kdim) {
  const int lane = threadIdx.x & (kWave - 1), r = lane & 15, kq = lane >> 4;
  const double* pr = p + r * pi;
  const double* qr = q + r * qj;
  for (int kc = 0; kc < kdim; kc += 32) {
    double a[8], b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = kc + 4 * t + kq;
      a[t] = (k < kdim && r < pm) ? pr[k * pk] : 0.0;
      b[t] = (k < kdim && r < qn) ? qr[k * qk] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) acc = mfma16(a[t], b[t], acc);
  }
}

__device__ int chol_inv_mfma(double* A, double* X, int n, double* lds) {
  double* T1 = lds;                 // diagonal tile, factored in place
  double* T0 = lds + kNb * kTl;     // its inverse
  double* tmp = lds + 2 * kNb * kTl;
  const int tid = threadIdx.x, wid = tid / kWave, lane = tid & (kWave - 1);
  const int r = lane & 15, rq = lane >> 4;
  const int nb = (n + kNb - 1) / kNb;
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = kb * kNb, kw = min(kNb, n - k0);
    for (int idx = tid; idx < kNb * kTl; idx += kBigThreads) {
      const int i = idx % kTl, j = idx / kTl;
      T1[idx] = (i < kw && j < kw && i >= j) ? A[k0 + i + (int64_t)(k0 + j) * n] : 0.0;
      T0[idx] = 0.0;
    }
    __syncthreads();
    const int f = chol_inplace<kBigThreads>(T1, kw, kTl);
    if (f) return k0 + f;
    trinv<kBigThreads>(T1, kTl, T0, kTl, kw, tmp);
    for (int idx = tid; idx < kw * kw; idx += kBigThreads) {
      const int i = idx % kw, j = idx / kw;
      X[k0 + i + (int64_t)(k0 + j) * n] = T0[i + j * kTl];   // zero above the diagonal
    }
    if (kb == nb - 1) break;
    // panel: A_Ik <- A_Ik X_kk^T, one 16-row strip per wave (kw = 64 here)
    const int p0 = k0 + kNb, nstrip = (n - p0 + 15) / 16;
    for (int s = wid; s < nstrip; s += kBigWaves) {
      const int i0 = p0 + 16 * s, im = min(16, n - i0);
      const double* ar = A + i0 + r + (int64_t)(k0 + (lane >> 4)) * n;
      d4_t acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = d4_t{0.0, 0.0, 0.0, 0.0};
      for (int kc = 0; kc < kNb; kc += 32) {
        double a[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] = r < im ? ar[(int64_t)(kc + 4 * t) * n] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int t = 0; t < 8; ++t)   // Q(k, j) = X_kk(j, k)
            acc[c] = mfma16(a[t], T0[16 * c + r + (kc + 4 * t + (lane >> 4)) * kTl], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (rq + 4 * v < im) A[i0 + rq + 4 * v + (int64_t)(k0 + 16 * c + r) * n] = acc[c][v];
    }
    __syncthreads();
    // trailing lower triangle, by 16 x 16 subtiles (I >= J strips)
    const int npair = nstrip * (nstrip + 1) / 2;
    for (int q = wid; q < npair; q += kBigWaves) {
      int I = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while ((I + 1) * (I + 2) / 2 <= q) ++I;
      while (I * (I + 1) / 2 > q) --I;
      const int J = q - I * (I + 1) / 2;
      const int i0 = p0 + 16 * I, j0 = p0 + 16 * J;
      const int im = min(16, n - i0), jm = min(16, n - j0);
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
      sub_mma(acc, A + i0 + (int64_t)k0 * n, 1, n, im, A + j0 + (int64_t)k0 * n, n, 1, jm, kNb);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rq + 4 * v < im && r < jm) A[i0 + rq + 4 * v + (int64_t)(j0 + r) * n] -= acc[v];
    }
    __syncthreads();
  }
  __syncthreads();
  // off-diagonal tiles of X, by anti-diagonals d = I - J
  for (int d = 1; d < nb; ++d) {
    const int nt = nb - d;   // tiles (J + d, J), J < nt
    // S_IJ = sum_{K=J}^{I-1} L_IK X_KJ into A(J-rows, I-cols), transposed
    for (int q = wid; q < nt * 16; q += kBigWaves) {
      const int jb = q / 16, sub = q % 16, ib = jb + d;
      const int i0 = ib * kNb + 16 * (sub / 4), j0 = jb * kNb + 16 * (sub % 4);
      if (i0 >= n) continue;
      const int im = min(16, n - i0);
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
      sub_mma(acc, A + i0 + (int64_t)(jb * kNb) * n, 1, n, im, X + jb * kNb + (int64_t)j0 * n, 1,
              n, 16, d * kNb);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rq + 4 * v < im) A[j0 + r + (int64_t)(i0 + rq + 4 * v) * n] = acc[v];
    }
    __syncthreads();
    // X_IJ = -X_II S_IJ; the mirrored upper tile of X is zeroed
    for (int q = wid; q < nt * 16; q += kBigWaves) {
      const int jb = q / 16, sub = q % 16, ib = jb + d;
      const int ii = ib * kNb, iw = min(kNb, n - ii);
      const int i0 = ii + 16 * (sub / 4), j0 = jb * kNb + 16 * (sub % 4);
      if (i0 >= n) continue;
      const int im = min(16, n - i0);
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
      sub_mma(acc, X + i0 + (int64_t)ii * n, 1, n, im, A + j0 + (int64_t)ii * n, n, 1, 16, iw);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rq + 4 * v < im) {
          X[i0 + rq + 4 * v + (int64_t)(j0 + r) * n] = -acc[v];
          X[j0 + r + (int64_t)(i0 + rq + 4 * v) * n] = 0.0;
        }
    }
    __syncthreads();
  }
  return 0;
}

__global__ __launch_bounds__(kBigThreads) void k_potrf_inv_big(const PotrfDesc* descs,
                                                               int32_t* info) {
  extern __shared__ double sm[];
  const PotrfDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (n == 0) return;
  const int tid = threadIdx.x;
  if (n <= kNb) {   // a small block of a launch with large ones: in LDS
    double* S = sm;
    double* X = sm + n * n;
    double* tmp = X + n * n;
    for (int idx = tid; idx < n * n; idx += kBigThreads) {
      const int i = idx % n, j = idx / n;
      S[idx] = i >= j ? d.A[i + (int64_t)j * d.lda] : 0.0;
    }
    __syncthreads();
    const int f = chol_inplace<kBigThreads>(S, n, n);
    if (f) {
      if (tid == 0) info[blockIdx.x] = f;
      for (int idx = tid; idx < n * n; idx += kBigThreads) d.X[idx] = 0.0;
      return;
    }
    trinv<kBigThreads>(S, n, X, n, n, tmp);
    for (int idx = tid; idx < n * n; idx += kBigThreads) d.X[idx] = X[idx];
  } else {
    // the panel's diagonal block (ld n) is dead after this call: factored in
    // place, its upper triangle used for the products S_IJ
    const int f = chol_inv_mfma(const_cast<double*>(d.A), d.X, n, sm);
    if (f) {
      if (tid == 0) info[blockIdx.x] = f;
      __syncthreads();
      for (int64_t idx = tid; idx < (int64_t)n * n; idx += kBigThreads) d.X[idx] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Cholesky + inverse of blocks of at most NM rows (NM = 32 or 64), one wave
// per block and the block in registers: lane i holds row i of the lower
// triangle, padded with the identity up to NM rows.  Column broadcasts go
// through NM doubles of LDS per wave; there are no workgroup barriers (the
// accesses of one wave to its LDS are in program order).
//  Cholesky, right-looking: at column j lane j's diagonal gives l_jj, the
//  lanes below scale their entry j and publish it, and every lane i updates
//  its entries c in (j, i] by l_ij l_cj.
//  Inverse in place, by columns from the last: with the lower-right block
//  already inverted, x_jj = 1 / l_jj and x_ij = -x_jj sum_{m=j+1..i} x_im l_mj.
// On breakdown the block's inverse is left zero (as in k_potrf_inv).
// ---------------------------------------------------------------------------
constexpr int kSmallWaves = 4;   // blocks (waves) per workgroup

__device__ __forceinline__ double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_d(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <class R, int NM>
__global__ __launch_bounds__(kSmallWaves * kWave) void k_potrf_inv_small(const PotrfDescT<R>* descs,
                                                                        int32_t count,
                                                                        int32_t* info) {
  __shared__ R colbuf[kSmallWaves][NM];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int b = blockIdx.x * kSmallWaves + w;
  if (b >= count) return;   // the whole wave leaves; no workgroup barriers follow
  const PotrfDescT<R> d = descs[b];
  const int n = d.n;
  if (n == 0) return;
  R* cb = colbuf[w];
  R row[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c)
    row[c] = (lane < n && c < n) ? (c <= lane ? d.A[lane + (int64_t)c * d.lda] : R(0))
                                 : (c == lane ? R(1) : R(0));
  int fail = 0;
  R rdl = 1;   // lane j: 1 / l_jj (1 in the identity padding)
#pragma unroll
  for (int j = 0; j < NM; ++j) {
    const R v = readlane_d(row[j], j);
    if (!(v > R(0))) {   // the same value in every lane
      fail = j + 1;
      break;
    }
    const R rs = rsqrt_nr(v);
    const R lij = lane > j ? row[j] * rs : (lane == j ? v * rs : R(0));
    if (lane == j) rdl = rs;   // 1 / l_jj, for the inverse
    if (lane >= j) row[j] = lij;
    if (lane < NM) cb[lane] = lij;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = j + 1; c < NM; ++c) {
      const R lcj = cb[c];
      if (lane >= c) row[c] = fma(-lij, lcj, row[c]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (fail) {
    if (lane == 0) info[b] = fail;
    for (int c = 0; c < n; ++c)
      if (lane < n) d.X[lane + (int64_t)c * n] = 0;
    return;
  }
#pragma unroll
  for (int j = NM - 1; j >= 0; --j) {
    if (lane < NM) cb[lane] = row[j];   // column j of L, before it is overwritten
    __builtin_amdgcn_wave_barrier();
    const R xjj = readlane_d(rdl, j);
    R acc = 0;
#pragma unroll
    for (int m = j + 1; m < NM; ++m)
      if (lane >= m) acc = fma(row[m], cb[m], acc);
    if (lane > j) row[j] = -xjj * acc;
    else if (lane == j) row[j] = xjj;
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int c = 0; c < NM; ++c)
    if (lane < n && c < n) d.X[lane + (int64_t)c * n] = row[c];
}

// ---------------------------------------------------------------------------
// Batched multi-term GEMM, 64x64 tile per workgroup: k-slabs of A and B staged
// in LDS, each wave a 32x32 quadrant as 2x2 matrix-core tiles of 16 x 16:
// FP64 (16 x 16 x 4 per instruction, R = double), FP32 (16 x 16 x 4, R =
// float) or BF16 (MODE = kGemmBf16: 16 x 16 x 16, FP32 accumulation), each
// FP32 operand split into two BF16 terms so that the products keep about 16
// bits (one BF16 product per pair broke the positive definiteness of the
// Schur complements of the 10^6-contrast diffusion matrices).
// ---------------------------------------------------------------------------
constexpr int kGemmThreads = 256;
constexpr int kGemmK = 16;

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

// FP32 16 x 16 x 4: operands as in mfma16; the accumulator gives lane l rows
// 4 (l / 16) + v, v = 0..3, of column l % 16.
__device__ __forceinline__ f4_t mfma16f(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// BF16 16 x 16 x 16: lane l supplies row l % 16 of the left factor at columns
// 4 (l / 16) + t and column l % 16 of the right factor at rows 4 (l / 16) + t,
// t = 0..3; FP32 accumulator laid out as in mfma16f.
__device__ __forceinline__ f4_t mfma16bf(s4_t a, s4_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// FP32 -> BF16, rounded to nearest (ties to even); the inputs are finite
__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(short h) {
  return __uint_as_float((unsigned)(unsigned short)h << 16);
}
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi): two BF16 terms carry
// 16 bits of x's mantissa
__device__ __forceinline__ void split_bf16(float x, short& hi, short& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - from_bf16(hi));
}

template <class R, int MODE>
__global__ __launch_bounds__(kGemmThreads, 8) void k_gemm(const GemmDescT<R>* descs,
                                                        const GemmTermT<R>* terms,
                                                        const TileRef* tiles) {
  constexpr bool kF64 = sizeof(R) == 8;
  using acc_t = typename std::conditional<kF64, d4_t, f4_t>::type;
  __shared__ R As[kGemmK][kGemmTile + 1];
  __shared__ R Bs[kGemmK][kGemmTile + 1];
  const TileRef t = tiles[blockIdx.x];
  const GemmDescT<R> d = descs[t.desc];
  const int i0 = t.ti * kGemmTile, j0 = t.tj * kGemmTile;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int wr = 32 * (w & 1), wc = 32 * (w >> 1), r = lane & 15, kq = lane >> 4;
  acc_t acc[2][2];
#pragma unroll
  for (int ri = 0; ri < 2; ++ri)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) acc[ri][ci] = acc_t{0, 0, 0, 0};
  for (int64_t term = d.term0; term < d.term1; ++term) {
    const GemmTermT<R> tm = terms[term];
    for (int k0 = 0; k0 < tm.k; k0 += kGemmK) {
      for (int e = threadIdx.x; e < kGemmTile * kGemmK; e += kGemmThreads) {
        int ii, kk;
        if (!d.transA) { ii = e % kGemmTile; kk = e / kGemmTile; }
        else { kk = e % kGemmK; ii = e / kGemmK; }
        const int gi = i0 + ii, gk = k0 + kk;
        R v = 0;
        if (gi < d.m && gk < tm.k)
          v = d.transA ? tm.A[gk + (int64_t)gi * tm.lda] : tm.A[gi + (int64_t)gk * tm.lda];
        As[kk][ii] = v;
      }
      for (int e = threadIdx.x; e < kGemmTile * kGemmK; e += kGemmThreads) {
        int jj, kk;
        if (!d.transB) { kk = e % kGemmK; jj = e / kGemmK; }
        else { jj = e % kGemmTile; kk = e / kGemmTile; }
        const int gj = j0 + jj, gk = k0 + kk;
        R v = 0;
        if (gj < d.n && gk < tm.k)
          v = d.transB ? tm.B[gj + (int64_t)gk * tm.ldb] : tm.B[gk + (int64_t)gj * tm.ldb];
        Bs[kk][jj] = v;
      }
      __syncthreads();
      if constexpr (MODE == kGemmBf16 && !kF64) {
        // each FP32 operand as a sum of two BF16 terms; the product keeps the
        // three terms above the 2^-16 level (hi hi, hi lo, lo hi)
        s4_t a0, a1, b0, b1, a0l, a1l, b0l, b1l;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int kk = 4 * kq + q;
          short h, l;
          split_bf16(As[kk][wr + r], h, l);
          a0[q] = h;
          a0l[q] = l;
          split_bf16(As[kk][wr + 16 + r], h, l);
          a1[q] = h;
          a1l[q] = l;
          split_bf16(Bs[kk][wc + r], h, l);
          b0[q] = h;
          b0l[q] = l;
          split_bf16(Bs[kk][wc + 16 + r], h, l);
          b1[q] = h;
          b1l[q] = l;
        }
        acc[0][0] = mfma16bf(a0, b0, acc[0][0]);
        acc[0][1] = mfma16bf(a0, b1, acc[0][1]);
        acc[1][0] = mfma16bf(a1, b0, acc[1][0]);
        acc[1][1] = mfma16bf(a1, b1, acc[1][1]);
        acc[0][0] = mfma16bf(a0, b0l, acc[0][0]);
        acc[0][1] = mfma16bf(a0, b1l, acc[0][1]);
        acc[1][0] = mfma16bf(a1, b0l, acc[1][0]);
        acc[1][1] = mfma16bf(a1, b1l, acc[1][1]);
        acc[0][0] = mfma16bf(a0l, b0, acc[0][0]);
        acc[0][1] = mfma16bf(a0l, b1, acc[0][1]);
        acc[1][0] = mfma16bf(a1l, b0, acc[1][0]);
        acc[1][1] = mfma16bf(a1l, b1, acc[1][1]);
      } else {
#pragma unroll
        for (int s4 = 0; s4 < kGemmK / 4; ++s4) {
          const int kk = 4 * s4 + kq;
          const R a0 = As[kk][wr + r], a1 = As[kk][wr + 16 + r];
          const R b0 = Bs[kk][wc + r], b1 = Bs[kk][wc + 16 + r];
          if constexpr (kF64) {
            acc[0][0] = mfma16(a0, b0, acc[0][0]);
            acc[0][1] = mfma16(a0, b1, acc[0][1]);
            acc[1][0] = mfma16(a1, b0, acc[1][0]);
            acc[1][1] = mfma16(a1, b1, acc[1][1]);
          } else {
            acc[0][0] = mfma16f(a0, b0, acc[0][0]);
            acc[0][1] = mfma16f(a0, b1, acc[0][1]);
            acc[1][0] = mfma16f(a1, b0, acc[1][0]);
            acc[1][1] = mfma16f(a1, b1, acc[1][1]);
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int ri = 0; ri < 2; ++ri)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int row = kF64 ? kq + 4 * v4 : 4 * kq + v4;
        const int gi = i0 + wr + 16 * ri + row, gj = j0 + wc + 16 * ci + r;
        if (gi < d.m && gj < d.n) {
          R v = R(d.alpha) * acc[ri][ci][v4];
          if (d.beta != 0.0) v = fma(R(d.beta), d.C[gi + (int64_t)gj * d.ldc], v);
          d.C[gi + (int64_t)gj * d.ldc] = v;
          if (d.C2) d.C2[gj + (int64_t)gi * d.ldc2] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// The same batched multi-term GEMM for blocks of at most 32 x 32 (the leaf
// steps' Schur targets are 5-30 rows): one wave per block, no LDS and no
// workgroup barriers.  The wave holds the block as 2 x 2 matrix-core tiles of
// 16 x 16 and reads its operands straight from global memory: in a 16-deep k
// step lane (r, q) = (l % 16, l / 16) loads rows k0 + 4q .. k0 + 4q + 3 of
// output row r's and column r's operand columns, and the t-th of the four
// products takes k = k0 + 4q + t (every k of the step once; the order of
// summation differs from the tile kernels'). refs[b].desc is the descriptor of
// wave b of the launch.
// ---------------------------------------------------------------------------
constexpr int kGemmSmallWaves = 4;

template <class R>
__global__ __launch_bounds__(kGemmSmallWaves * kWave) void k_gemm_small(const GemmDescT<R>* descs,
                                                                      const GemmTermT<R>* terms,
                                                                      const TileRef* refs,
                                                                      int64_t count) {
  constexpr bool kF64 = sizeof(R) == 8;
  using acc_t = typename std::conditional<kF64, d4_t, f4_t>::type;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t b = (int64_t)blockIdx.x * kGemmSmallWaves + threadIdx.x / kWave;
  if (b >= count) return;   // the whole wave leaves; no workgroup barriers
  const GemmDescT<R> d = descs[refs[b].desc];
  const int r = lane & 15, q = lane >> 4;
  const bool one = d.m <= 16 && d.n <= 16;
  acc_t acc[2][2];
#pragma unroll
  for (int ri = 0; ri < 2; ++ri)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) acc[ri][ci] = acc_t{0, 0, 0, 0};
  for (int64_t term = d.term0; term < d.term1; ++term) {
    const GemmTermT<R> tm = terms[term];
    for (int k0 = 0; k0 < tm.k; k0 += 16) {
      R a[2][4], bv[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 16 * h + r;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int k = k0 + 4 * q + t;
          const bool in_a = i < d.m && k < tm.k, in_b = i < d.n && k < tm.k;
          a[h][t] = in_a ? (d.transA ? tm.A[k + (int64_t)i * tm.lda] : tm.A[i + (int64_t)k * tm.lda])
                         : R(0);
          bv[h][t] = in_b ? (d.transB ? tm.B[i + (int64_t)k * tm.ldb] : tm.B[k + (int64_t)i * tm.ldb])
                          : R(0);
        }
      }
      if (one) {   // a block of at most 16 x 16: one matrix-core tile
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if constexpr (kF64) acc[0][0] = mfma16(a[0][t], bv[0][t], acc[0][0]);
          else acc[0][0] = mfma16f(a[0][t], bv[0][t], acc[0][0]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri)
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
              if constexpr (kF64) acc[ri][ci] = mfma16(a[ri][t], bv[ci][t], acc[ri][ci]);
              else acc[ri][ci] = mfma16f(a[ri][t], bv[ci][t], acc[ri][ci]);
            }
      }
    }
  }
#pragma unroll
  for (int ri = 0; ri < 2; ++ri)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int row = kF64 ? q + 4 * v4 : 4 * q + v4;
        const int gi = 16 * ri + row, gj = 16 * ci + r;
        if (gi < d.m && gj < d.n) {
          R v = R(d.alpha) * acc[ri][ci][v4];
          if (d.beta != 0.0) v = fma(R(d.beta), d.C[gi + (int64_t)gj * d.ldc], v);
          d.C[gi + (int64_t)gj * d.ldc] = v;
          if (d.C2) d.C2[gj + (int64_t)gi * d.ldc2] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// The same batched multi-term GEMM over 128 x 128 output tiles, for launches
// of large blocks: each of the four waves owns a 64 x 64 quadrant as 4 x 4
// matrix-core tiles of 16 x 16 (16 instructions per 4-deep k step against 4
// for the 64-tile kernel, for the same two LDS operand loads per subtile row
// or column), and the k-slabs are double buffered: the next slab's global
// loads are issued into registers before the current slab's products, and
// stored into the other LDS buffer after them, so one barrier per slab
// separates the two and the global latency hides behind the matrix cores.
// ---------------------------------------------------------------------------
constexpr int kG2 = 128;                         // output tile
constexpr int kG2Per = kG2 * kGemmK / kGemmThreads;   // slab elements per thread and operand

template <class R, int MODE>
__global__ __launch_bounds__(kGemmThreads, 2) void k_gemm128(const GemmDescT<R>* descs,
                                                           const GemmTermT<R>* terms,
                                                           const TileRef* tiles) {
  constexpr bool kF64 = sizeof(R) == 8;
  using acc_t = typename std::conditional<kF64, d4_t, f4_t>::type;
  __shared__ R As[2][kGemmK][kG2 + 1];
  __shared__ R Bs[2][kGemmK][kG2 + 1];
  const TileRef t = tiles[blockIdx.x];
  const GemmDescT<R> d = descs[t.desc];
  const int i0 = t.ti * kG2, j0 = t.tj * kG2;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int wr = 64 * (w & 1), wc = 64 * (w >> 1), r = lane & 15, kq = lane >> 4;
  acc_t acc[4][4];
#pragma unroll
  for (int ri = 0; ri < 4; ++ri)
#pragma unroll
    for (int ci = 0; ci < 4; ++ci) acc[ri][ci] = acc_t{0, 0, 0, 0};
  // slab (term, k0) -> registers
  R ra[kG2Per], rb[kG2Per];
  auto fetch = [&](int64_t term, int k0) {
    const GemmTermT<R> tm = terms[term];
#pragma unroll
    for (int q = 0; q < kG2Per; ++q) {
      const int e = threadIdx.x + q * kGemmThreads;
      int ii, kk;
      if (!d.transA) { ii = e % kG2; kk = e / kG2; }
      else { kk = e % kGemmK; ii = e / kGemmK; }
      const int gi = i0 + ii, gk = k0 + kk;
      ra[q] = (gi < d.m && gk < tm.k)
                  ? (d.transA ? tm.A[gk + (int64_t)gi * tm.lda] : tm.A[gi + (int64_t)gk * tm.lda])
                  : R(0);
      int jj, kb;
      if (!d.transB) { kb = e % kGemmK; jj = e / kGemmK; }
      else { jj = e % kG2; kb = e / kG2; }
      const int gj = j0 + jj, gk2 = k0 + kb;
      rb[q] = (gj < d.n && gk2 < tm.k)
                  ? (d.transB ? tm.B[gj + (int64_t)gk2 * tm.ldb] : tm.B[gk2 + (int64_t)gj * tm.ldb])
                  : R(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kG2Per; ++q) {
      const int e = threadIdx.x + q * kGemmThreads;
      if (!d.transA) As[buf][e / kG2][e % kG2] = ra[q];
      else As[buf][e % kGemmK][e / kGemmK] = ra[q];
      if (!d.transB) Bs[buf][e % kGemmK][e / kGemmK] = rb[q];
      else Bs[buf][e / kG2][e % kG2] = rb[q];
    }
  };
  int64_t term = d.term0;
  int k0 = 0;
  if (term >= d.term1) return;
  while (term < d.term1 && terms[term].k == 0) ++term;
  int cur = 0;
  if (term < d.term1) {
    fetch(term, 0);
    stash(0);
  }
  __syncthreads();
  while (term < d.term1) {
    // the slab after (term, k0)
    int64_t nterm = term;
    int nk0 = k0 + kGemmK;
    if (nk0 >= terms[term].k) {
      nk0 = 0;
      ++nterm;
      while (nterm < d.term1 && terms[nterm].k == 0) ++nterm;
    }
    const bool more = nterm < d.term1;
    if (more) fetch(nterm, nk0);
    if constexpr (MODE == kGemmBf16 && !kF64) {
      s4_t ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * kq + q;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          short h, l;
          split_bf16(As[cur][kk][wr + 16 * x + r], h, l);
          ah[x][q] = h;
          al[x][q] = l;
          split_bf16(Bs[cur][kk][wc + 16 * x + r], h, l);
          bh[x][q] = h;
          bl[x][q] = l;
        }
      }
#pragma unroll
      for (int ri = 0; ri < 4; ++ri)
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) {
          acc[ri][ci] = mfma16bf(ah[ri], bh[ci], acc[ri][ci]);
          acc[ri][ci] = mfma16bf(ah[ri], bl[ci], acc[ri][ci]);
          acc[ri][ci] = mfma16bf(al[ri], bh[ci], acc[ri][ci]);
        }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < kGemmK / 4; ++s4) {
        const int kk = 4 * s4 + kq;
        R a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          a[x] = As[cur][kk][wr + 16 * x + r];
          b[x] = Bs[cur][kk][wc + 16 * x + r];
        }
#pragma unroll
        for (int ri = 0; ri < 4; ++ri)
#pragma unroll
          for (int ci = 0; ci < 4; ++ci) {
            if constexpr (kF64) acc[ri][ci] = mfma16(a[ri], b[ci], acc[ri][ci]);
            else acc[ri][ci] = mfma16f(a[ri], b[ci], acc[ri][ci]);
          }
      }
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
    cur ^= 1;
    term = nterm;
    k0 = nk0;
  }
#pragma unroll
  for (int ri = 0; ri < 4; ++ri)
#pragma unroll
    for (int ci = 0; ci < 4; ++ci)
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const int row = kF64 ? kq + 4 * v4 : 4 * kq + v4;
        const int gi = i0 + wr + 16 * ri + row, gj = j0 + wc + 16 * ci + r;
        if (gi < d.m && gj < d.n) {
          R v = R(d.alpha) * acc[ri][ci][v4];
          if (d.beta != 0.0) v = fma(R(d.beta), d.C[gi + (int64_t)gj * d.ldc], v);
          d.C[gi + (int64_t)gj * d.ldc] = v;
          if (d.C2) d.C2[gj + (int64_t)gi * d.ldc2] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Early-stopping column-pivoted Householder QR, one interface per workgroup.
// The coupling W (a x k) is copied transposed into the workspace Yt
// (element (i, c) at Yt[c + i*kmax]), so one thread owns one column: the
// reflector's dot product, the rank-1 update and the exact trailing norm of
// the column need no cross-lane reduction, and the 64 lanes of a wave touch
// 64 consecutive columns of a row (coalesced).  The first kQrCache rows of the
// trailing column stay in registers between the dot and the update pass.
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 1024;
constexpr int kQrWaves = kQrThreads / kWave;
constexpr int kQrCache = 8;    // rows of a column kept in registers between passes
constexpr int kQrUnroll = 8;   // independent loads in flight per thread

template <class R>
__global__ __launch_bounds__(kQrThreads) void k_cpqr(const CpqrDescT<R>* descs, const CpqrNbrT<R>* nbrs,
                                                      int32_t* n_cur, int32_t* out_r,
                                                      int32_t* out_r2, int32_t* out_k,
                                                      double eps, double eps_stop, int32_t max_k) {
  extern __shared__ __align__(16) char smraw[];
  R* sm = reinterpret_cast<R*>(smraw);
  __shared__ R redd[kQrWaves];
  __shared__ int redi[kQrWaves];
  const CpqrDescT<R> d = descs[blockIdx.x];
  const int a = d.a;
  const int64_t K = d.kmax;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  R* nrm2 = sm;
  R* v = sm + max_k;
  R* __restrict__ Yt = d.Y;

  // gather W^T: the neighbours' blocks (p, w) with their current widths
  int k = 0;
  for (int64_t e = d.nb0; e < d.nb1; ++e) {
    const CpqrNbrT<R> nb = nbrs[e];
    const int wc = n_cur[nb.w];
    const R* src = d.panel + nb.col * a;
    for (int idx = tid; idx < a * wc; idx += kQrThreads) {
      const int c = idx % wc, i = idx / wc;
      Yt[(k + c) + i * K] = src[i + (int64_t)c * a];
    }
    k += wc;
  }
  __syncthreads();
  for (int c = tid; c < k; c += kQrThreads) {
    const R* col = Yt + c;
    R s = 0.0;
    int i = 0;
    for (; i + kQrUnroll <= a; i += kQrUnroll) {
      R y[kQrUnroll];
#pragma unroll
      for (int u = 0; u < kQrUnroll; ++u) y[u] = col[(i + u) * K];
#pragma unroll
      for (int u = 0; u < kQrUnroll; ++u) s = fma(y[u], y[u], s);
    }
    for (; i < a; ++i) s = fma(col[i * K], col[i * K], s);
    nrm2[c] = s;
  }
  __syncthreads();

  int r = -1;
  int j = 0;
  R R00 = 0.0;
  const int jmax = min(a, k);
  for (; j < jmax; ++j) {
    R m = -1.0;
    for (int c = tid; c < k; c += kQrThreads) m = fmax(m, nrm2[c]);
    m = wave_max(m);
    if (lane == 0) redd[wid] = m;
    __syncthreads();
    R M = redd[0];
#pragma unroll
    for (int w = 1; w < kQrWaves; ++w) M = fmax(M, redd[w]);
    if (M < 0.0) break;
    const R thr = M * R(1.0 - PivotTie<R>::rtol);
    int cand = INT_MAX;
    for (int c = tid; c < k; c += kQrThreads)
      if (nrm2[c] >= 0.0 && nrm2[c] >= thr) { cand = c; break; }
    cand = wave_min_int(cand);
    if (lane == 0) redi[wid] = cand;
    __syncthreads();
    int C = redi[0];
#pragma unroll
    for (int w = 1; w < kQrWaves; ++w) C = min(C, redi[w]);
    const R nrm = sqrt(nrm2[C]);
    if (j == 0) R00 = nrm;
    if (nrm == 0.0 || nrm < eps_stop * R00) break;
    if (r < 0 && nrm < eps * R00) r = j;
    const R alpha = Yt[C + j * K];
    const R beta = alpha >= R(0) ? -nrm : nrm;
    const R denom = alpha - beta;
    const R tau = (beta - alpha) / beta;
    for (int i = tid; i < a; i += kQrThreads) {
      const R vi = i < j ? R(0) : (i == j ? R(1) : Yt[C + i * K] / denom);
      v[i] = vi;
      d.V[i + (int64_t)j * a] = vi;
    }
    if (tid == 0) d.tau[j] = tau;
    __syncthreads();
    for (int c = tid; c < k; c += kQrThreads) {
      if (c == C || nrm2[c] < 0.0) continue;
      R* __restrict__ col = Yt + c;
      R cache[kQrCache];
      R w0 = 0.0, w1 = 0.0;
#pragma unroll
      for (int t = 0; t < kQrCache; ++t) {
        const int i = j + t;
        cache[t] = i < a ? col[i * K] : R(0);
      }
#pragma unroll
      for (int t = 0; t < kQrCache; ++t) w0 = fma(j + t < a ? v[j + t] : R(0), cache[t], w0);
      int i = j + kQrCache;
      for (; i + kQrUnroll <= a; i += kQrUnroll) {
        R y[kQrUnroll];
#pragma unroll
        for (int u = 0; u < kQrUnroll; ++u) y[u] = col[(i + u) * K];
#pragma unroll
        for (int u = 0; u < kQrUnroll; ++u) w1 = fma(v[i + u], y[u], w1);
      }
      for (; i < a; ++i) w1 = fma(v[i], col[i * K], w1);
      const R w = (w0 + w1) * tau;
      R s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int t = 0; t < kQrCache; ++t) {
        const int ii = j + t;
        if (ii < a) {
          const R y = fma(-w, v[ii], cache[t]);
          col[ii * K] = y;
          if (t > 0) s0 = fma(y, y, s0);
        }
      }
      i = j + kQrCache;
      for (; i + kQrUnroll <= a; i += kQrUnroll) {
        R y[kQrUnroll];
#pragma unroll
        for (int u = 0; u < kQrUnroll; ++u) y[u] = col[(i + u) * K];
#pragma unroll
        for (int u = 0; u < kQrUnroll; ++u) {
          y[u] = fma(-w, v[i + u], y[u]);
          s1 = fma(y[u], y[u], s1);
        }
#pragma unroll
        for (int u = 0; u < kQrUnroll; ++u) col[(i + u) * K] = y[u];
      }
      for (; i < a; ++i) {
        const R y = fma(-w, v[i], col[i * K]);
        col[i * K] = y;
        s1 = fma(y, y, s1);
      }
      nrm2[c] = s0 + s1;
    }
    for (int i = j + tid; i < a; i += kQrThreads) Yt[C + i * K] = i == j ? beta : R(0);
    if (tid == 0) nrm2[C] = -1.0;
    __syncthreads();
  }
  const int nref = j;
  if (r < 0) r = nref;

  // coarse rows back into p's panel and, transposed, into the neighbours' panels
  int kk = 0;
  for (int64_t e = d.nb0; e < d.nb1; ++e) {
    const CpqrNbrT<R> nb = nbrs[e];
    const int wc = n_cur[nb.w];
    for (int idx = tid; idx < r * wc; idx += kQrThreads) {
      const int c = idx % wc, i = idx / wc;
      const R y = Yt[(kk + c) + i * K];
      d.panel[i + (nb.col + c) * a] = y;
      nb.blk_wp[c + (int64_t)i * nb.ldw] = y;
    }
    kk += wc;
  }
  for (int idx = tid; idx < r * r; idx += kQrThreads) {
    const int i = idx % r, c = idx / r;
    d.panel[i + (d.diag_col + c) * a] = i == c ? R(1) : R(0);
  }
  if (tid == 0) {
    out_k[d.p] = k;
    out_r[d.p] = r;
    out_r2[d.p] = nref;
  }
  __syncthreads();
  if (tid == 0) n_cur[d.p] = r;
}

// Triangular factor T of the compact WY form Q = H_0 H_1 ... H_{n-1} = I - V T V^T
// of one interface's n reflectors.  T is upper triangular with
// T^{-1} = diag(1/tau) + (strict upper part of V^T V), so column j follows from
// the earlier ones: T_jj = tau_j, T_{0:j,j} = -tau_j T_{0:j,0:j} (V^T V)_{0:j,j}.
// On entry T holds V^T V in its lower triangle.  The work array A (n x n,
// column-major) holds T on and above the diagonal and V^T V below it; it lives
// in LDS when n <= kWyLdsN, else in T itself.  Row sums use 8-lane groups.
template <class R, bool kInLds>
__global__ __launch_bounds__(kWyThreads) void k_wy_t(const WyDescT<R>* descs) {
  extern __shared__ __align__(16) char smraw[];
  R* lds = reinterpret_cast<R*>(smraw);
  const WyDescT<R> d = descs[blockIdx.x];
  const int n = d.n;
  if (n <= 0 || (n <= kWyLdsN) != kInLds) return;
  // n > kWyLdsN: this recurrence only when some tau is 0 (T^-1 does not exist);
  // otherwise k_wy_t_inv inverts T^-1 by tiles
  if (!kInLds) {
    bool zero = false;
    for (int j = threadIdx.x; j < n; j += kWyThreads) zero = zero || d.tau[j] == R(0);
    if (!__syncthreads_or(zero)) return;
  }
  R* A = kInLds ? lds : d.T;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int grp = lane >> 3, r8 = lane & 7;
  constexpr int kGroups = kWyThreads / 8;
  if (kInLds)
    for (int64_t idx = tid; idx < (int64_t)n * n; idx += kWyThreads) {
      const int i = (int)(idx % n), c = (int)(idx / n);
      if (i > c) A[idx] = d.T[idx];
    }
  for (int j = tid; j < n; j += kWyThreads) A[j + (int64_t)j * n] = d.tau[j];
  __syncthreads();
  for (int j = 1; j < n; ++j) {
    const R tj = d.tau[j];
    for (int ib = wid * 8; ib < j; ib += kGroups) {   // wave-uniform bound
      const int i = ib + grp;
      R acc = 0;
      if (i < j)
        for (int q = i + r8; q < j; q += 8)
          acc = fma(A[i + (int64_t)q * n], A[j + (int64_t)q * n], acc);
      acc = group8_sum(acc);
      if (i < j && r8 == 0) A[i + (int64_t)j * n] = -tj * acc;
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += kWyThreads) {
    const int i = (int)(idx % n), c = (int)(idx / n);
    d.T[idx] = i <= c ? A[idx] : R(0);
  }
}

// T of a compact WY form with more than kWyLdsN reflectors, all tau nonzero:
// T^{-1} = diag(1/tau) + (strict upper part of V^T V) is upper triangular, so
// T = X^T with X the inverse of the lower triangular L = diag(1/tau) + (strict
// lower part of V^T V), by 64x64 tiles (trinv on the diagonal tiles, block
// forward substitution below).  On entry T holds V^T V in its lower triangle;
// L is formed in place there, X goes to the scratch d.X.  LDS: four 64x65
// tiles.
template <class R>
__global__ __launch_bounds__(kPotrfThreads) void k_wy_t_inv(const WyDescT<R>* descs) {
  extern __shared__ __align__(16) char smraw[];
  R* sm = reinterpret_cast<R*>(smraw);
  const WyDescT<R> d = descs[blockIdx.x];
  const int n = d.n;
  if (n <= kWyLdsN) return;
  bool zero = false;
  for (int j = threadIdx.x; j < n; j += kPotrfThreads) zero = zero || d.tau[j] == R(0);
  if (__syncthreads_or(zero)) return;   // k_wy_t<false> takes it
  for (int j = threadIdx.x; j < n; j += kPotrfThreads) d.T[j + (int64_t)j * n] = R(1) / d.tau[j];
  __syncthreads();
  R* T0 = sm;
  R* T1 = sm + kNb * kTl;
  R* tmp = sm + 3 * kNb * kTl;
  const int nb = (n + kNb - 1) / kNb;
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = kb * kNb, kw = min(kNb, n - k0);
    tile_load(T1, d.T + k0 + (int64_t)k0 * n, n, kw, kw);
    for (int idx = threadIdx.x; idx < kNb * kTl; idx += kPotrfThreads) T0[idx] = 0;
    __syncthreads();
    trinv<kPotrfThreads>(T1, kTl, T0, kTl, kw, tmp);
    for (int idx = threadIdx.x; idx < kw * kw; idx += kPotrfThreads) {
      const int i = idx % kw, j = idx / kw;
      d.X[k0 + i + (int64_t)(k0 + j) * n] = i >= j ? T0[i + j * kTl] : R(0);
    }
    __syncthreads();
  }
  lower_inv_offdiag(d.T, d.X, n, sm);
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += kPotrfThreads) {
    const int i = (int)(idx % n), c = (int)(idx / n);
    d.T[idx] = i <= c ? d.X[c + (int64_t)i * n] : R(0);
  }
}

template <class R>
__global__ void k_fill(R* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = R(v);
}

template <class R>
__global__ void k_scatter(const double* vals, const int64_t* dest, int64_t nnz, R* panels) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    panels[dest[e]] = R(vals[e]);
}

template <class S, class D>
__global__ __launch_bounds__(256) void k_copy(const CopyDescT<S, D>* descs) {
  const CopyDescT<S, D> d = descs[blockIdx.x];
  const int m = d.m;
  if ((int64_t)d.m * d.n <= INT_MAX) {
    // 32-bit index arithmetic (a 64-bit division per element cost more than
    // the copy itself)
    const int mn = d.m * d.n;
    for (int idx = threadIdx.x; idx < mn; idx += blockDim.x) {
      const int j = idx / m, i = idx - j * m;
      d.dst[i + (int64_t)j * d.ldd] = D(d.src[i + (int64_t)j * d.lds]);
    }
  } else {
    for (int j = 0; j < d.n; ++j)
      for (int i = threadIdx.x; i < m; i += blockDim.x)
        d.dst[i + (int64_t)j * d.ldd] = D(d.src[i + (int64_t)j * d.lds]);
  }
}

inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

template <class R>
void launch_fill(R* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<R>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

template <class R>
void launch_scatter(const double* vals, const int64_t* dest, int64_t nnz, R* panels, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_scatter<R>, dim3(grid_for(nnz, 256)), dim3(256), 0, s, vals, dest, nnz,
                     panels);
}

template <class R>
void launch_potrf_inv(const PotrfDescT<R>* d, int32_t count, int32_t max_n, int32_t* info,
                      hipStream_t s) {
  if (count <= 0) return;
  if (max_n <= 64) {   // one wave per block, in registers
    const dim3 grid((unsigned)((count + kSmallWaves - 1) / kSmallWaves)), block(kSmallWaves * kWave);
    if (max_n <= 32) hipLaunchKernelGGL((k_potrf_inv_small<R, 32>), grid, block, 0, s, d, count, info);
    else hipLaunchKernelGGL((k_potrf_inv_small<R, 64>), grid, block, 0, s, d, count, info);
    return;
  }
  launch_potrf_blocks(d, count, max_n, info, s);
}

template <class R>
void launch_potrf_blocks(const PotrfDescT<R>* d, int32_t count, int32_t max_n, int32_t* info,
                         hipStream_t s) {
  if (count <= 0) return;
  if (max_n > kNb) {   // two 64x65 tiles and the inverse's products
    if constexpr (sizeof(R) == 8) {
      const size_t lds = ((size_t)2 * kNb * kTl + 768) * sizeof(double);
      hipLaunchKernelGGL(k_potrf_inv_big, dim3(count), dim3(kBigThreads), lds, s, d, info);
    } else {
      __builtin_trap();   // unreachable: the FP32 forms factor such blocks in FP64
    }
    return;
  }
  // the block, its inverse and the inverse's products in LDS
  const size_t lds = ((size_t)2 * max_n * max_n + 768) * sizeof(R);
  hipLaunchKernelGGL(k_potrf_inv<R>, dim3(count), dim3(kPotrfThreads), lds, s, d, info);
}

template <class R>
void launch_gemm(const GemmDescT<R>* d, const GemmTermT<R>* t, const TileRef* tiles, int64_t ntiles,
                 GemmMode mode, int tile, hipStream_t s) {
  if (ntiles <= 0) return;
  const dim3 grid((unsigned)ntiles), block(kGemmThreads);
  if constexpr (sizeof(R) == 4) {
    if (mode == kGemmBf16) {
      if (tile == kG2) hipLaunchKernelGGL((k_gemm128<R, kGemmBf16>), grid, block, 0, s, d, t, tiles);
      else hipLaunchKernelGGL((k_gemm<R, kGemmBf16>), grid, block, 0, s, d, t, tiles);
      return;
    }
  }
  if (tile == kG2) hipLaunchKernelGGL((k_gemm128<R, kGemmNative>), grid, block, 0, s, d, t, tiles);
  else hipLaunchKernelGGL((k_gemm<R, kGemmNative>), grid, block, 0, s, d, t, tiles);
}

template <class R>
void launch_gemm_small(const GemmDescT<R>* d, const GemmTermT<R>* t, const TileRef* refs,
                       int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const dim3 grid((unsigned)((count + kGemmSmallWaves - 1) / kGemmSmallWaves));
  hipLaunchKernelGGL(k_gemm_small<R>, grid, dim3(kGemmSmallWaves * kWave), 0, s, d, t, refs, count);
}

template <class R>
void launch_cpqr(const CpqrDescT<R>* d, const CpqrNbrT<R>* nb, int32_t count, int32_t* n_cur,
                 int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps, double eps_stop,
                 int32_t max_a, int32_t max_k, hipStream_t s) {
  if (count <= 0) return;
  size_t lds = ((size_t)max_k + max_a) * sizeof(R);
  hipLaunchKernelGGL(k_cpqr<R>, dim3(count), dim3(kQrThreads), lds, s, d, nb, n_cur, out_r, out_r2,
                     out_k, eps, eps_stop, max_k);
}

template <class R>
void launch_wy_t(const WyDescT<R>* d, int32_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_wy_t<R, true>), dim3(count), dim3(kWyThreads),
                     (size_t)kWyLdsN * kWyLdsN * sizeof(R), s, d);
  hipLaunchKernelGGL((k_wy_t<R, false>), dim3(count), dim3(kWyThreads), 0, s, d);
  hipLaunchKernelGGL(k_wy_t_inv<R>, dim3(count), dim3(kPotrfThreads),
                     (size_t)4 * kNb * kTl * sizeof(R), s, d);
}

template <class S, class D>
void launch_copy(const CopyDescT<S, D>* d, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_copy<S, D>), dim3((unsigned)count), dim3(256), 0, s, d);
}

#define SPAND_FACTOR_INST(R)                                                                      \
  template void launch_fill<R>(R*, int64_t, double, hipStream_t);                                 \
  template void launch_scatter<R>(const double*, const int64_t*, int64_t, R*, hipStream_t);       \
  template void launch_potrf_inv<R>(const PotrfDescT<R>*, int32_t, int32_t, int32_t*, hipStream_t); \
  template void launch_potrf_blocks<R>(const PotrfDescT<R>*, int32_t, int32_t, int32_t*,          \
                                       hipStream_t);                                              \
  template void launch_gemm<R>(const GemmDescT<R>*, const GemmTermT<R>*, const TileRef*, int64_t, \
                               GemmMode, int, hipStream_t);                                       \
  template void launch_gemm_small<R>(const GemmDescT<R>*, const GemmTermT<R>*, const TileRef*,    \
                                     int64_t, hipStream_t);                                       \
  template void launch_cpqr<R>(const CpqrDescT<R>*, const CpqrNbrT<R>*, int32_t, int32_t*,        \
                               int32_t*, int32_t*, int32_t*, double, double, int32_t, int32_t,    \
                               hipStream_t);                                                      \
  template void launch_wy_t<R>(const WyDescT<R>*, int32_t, hipStream_t);
SPAND_FACTOR_INST(double)
SPAND_FACTOR_INST(float)
#undef SPAND_FACTOR_INST
template void launch_copy<double, double>(const CopyDescT<double, double>*, int64_t, hipStream_t);
template void launch_copy<float, float>(const CopyDescT<float, float>*, int64_t, hipStream_t);
template void launch_copy<float, double>(const CopyDescT<float, double>*, int64_t, hipStream_t);
template void launch_copy<double, float>(const CopyDescT<double, float>*, int64_t, hipStream_t);

}  // namespace spand
