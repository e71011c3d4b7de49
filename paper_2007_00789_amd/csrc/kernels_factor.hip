// HIP kernels of the factorization (FP64, gfx950).
//
//  k_potrf_inv : batched uneven Cholesky + triangular inverse, one workgroup
//                per block; blocks up to 128 rows live in LDS, larger ones are
//                factored in place in global memory.
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

#include "device.h"

namespace spand {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
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

// ---------------------------------------------------------------------------
// Cholesky + inverse of the lower factor.  Column-oriented right-looking
// factorization; the inverse is formed in place column by column from the
// right (X_jj = 1/L_jj, X_{j+1:,j} = -X_jj X_{j+1:,j+1:} L_{j+1:,j}).
// S: n x n column-major (LDS or global), tmp: n doubles of LDS.
// Returns 0 or the 1-based column of the first non-positive pivot.
// ---------------------------------------------------------------------------
template <int NT>
__device__ int chol_inv_inplace(double* S, int n, int ld, double* tmp, int* flag) {
  const int tid = threadIdx.x;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double v = S[j + (int64_t)j * ld];
      if (!(v > 0.0)) *flag = j + 1;
      else S[j + (int64_t)j * ld] = sqrt(v);
    }
    __syncthreads();
    if (*flag) return *flag;
    const double djj = S[j + (int64_t)j * ld];
    for (int i = j + 1 + tid; i < n; i += NT) S[i + (int64_t)j * ld] /= djj;
    __syncthreads();
    const int m = n - j - 1;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int ii = idx % m, cc = idx / m;
      if (ii >= cc) {
        const int i = j + 1 + ii, c = j + 1 + cc;
        S[i + (int64_t)c * ld] -= S[i + (int64_t)j * ld] * S[c + (int64_t)j * ld];
      }
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < n; i += NT) tmp[i] = S[i + (int64_t)j * ld];
    __syncthreads();
    const double inv = 1.0 / S[j + (int64_t)j * ld];
    for (int i = j + 1 + tid; i < n; i += NT) {
      double acc = 0.0;
      for (int m2 = j + 1; m2 <= i; ++m2) acc = fma(S[i + (int64_t)m2 * ld], tmp[m2], acc);
      S[i + (int64_t)j * ld] = -inv * acc;
    }
    __syncthreads();
    if (tid == 0) S[j + (int64_t)j * ld] = inv;
    __syncthreads();
  }
  return 0;
}

constexpr int kPotrfThreads = 256;

__global__ __launch_bounds__(kPotrfThreads) void k_potrf_inv(const PotrfDesc* descs, int32_t* info) {
  extern __shared__ double sm[];
  __shared__ int flag;
  const PotrfDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (n == 0) return;
  const int tid = threadIdx.x;
  if (n <= kPotrfLdsMax) {
    double* S = sm;
    double* tmp = sm + n * n;
    for (int idx = tid; idx < n * n; idx += kPotrfThreads) {
      const int i = idx % n, j = idx / n;
      S[idx] = i >= j ? d.A[i + (int64_t)j * d.lda] : 0.0;
    }
    __syncthreads();
    const int f = chol_inv_inplace<kPotrfThreads>(S, n, n, tmp, &flag);
    if (f) {
      if (tid == 0) info[blockIdx.x] = f;
      return;
    }
    for (int idx = tid; idx < n * n; idx += kPotrfThreads) d.X[idx] = S[idx];
  } else {
    for (int64_t idx = tid; idx < (int64_t)n * n; idx += kPotrfThreads) {
      const int i = (int)(idx % n), j = (int)(idx / n);
      d.X[idx] = i >= j ? d.A[i + (int64_t)j * d.lda] : 0.0;
    }
    __syncthreads();
    const int f = chol_inv_inplace<kPotrfThreads>(d.X, n, n, sm, &flag);
    if (f && tid == 0) info[blockIdx.x] = f;
  }
}

// ---------------------------------------------------------------------------
// Batched multi-term GEMM, 64x64 tile per workgroup, 4x4 per thread.
// ---------------------------------------------------------------------------
constexpr int kGemmThreads = 256;
constexpr int kGemmK = 16;

__global__ __launch_bounds__(kGemmThreads) void k_gemm(const GemmDesc* descs, const GemmTerm* terms,
                                                        const TileRef* tiles) {
  __shared__ double As[kGemmK][kGemmTile + 1];
  __shared__ double Bs[kGemmK][kGemmTile + 1];
  const TileRef t = tiles[blockIdx.x];
  const GemmDesc d = descs[t.desc];
  const int i0 = t.ti * kGemmTile, j0 = t.tj * kGemmTile;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int64_t term = d.term0; term < d.term1; ++term) {
    const GemmTerm tm = terms[term];
    for (int k0 = 0; k0 < tm.k; k0 += kGemmK) {
      for (int e = threadIdx.x; e < kGemmTile * kGemmK; e += kGemmThreads) {
        int ii, kk;
        if (!d.transA) { ii = e % kGemmTile; kk = e / kGemmTile; }
        else { kk = e % kGemmK; ii = e / kGemmK; }
        const int gi = i0 + ii, gk = k0 + kk;
        double v = 0.0;
        if (gi < d.m && gk < tm.k)
          v = d.transA ? tm.A[gk + (int64_t)gi * tm.lda] : tm.A[gi + (int64_t)gk * tm.lda];
        As[kk][ii] = v;
      }
      for (int e = threadIdx.x; e < kGemmTile * kGemmK; e += kGemmThreads) {
        int jj, kk;
        if (!d.transB) { kk = e % kGemmK; jj = e / kGemmK; }
        else { jj = e % kGemmTile; kk = e / kGemmTile; }
        const int gj = j0 + jj, gk = k0 + kk;
        double v = 0.0;
        if (gj < d.n && gk < tm.k)
          v = d.transB ? tm.B[gj + (int64_t)gk * tm.ldb] : tm.B[gk + (int64_t)gj * tm.ldb];
        Bs[kk][jj] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kGemmK; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = As[kk][tx + 16 * r];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = Bs[kk][ty + 16 * c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gi = i0 + tx + 16 * r, gj = j0 + ty + 16 * c;
      if (gi < d.m && gj < d.n) {
        double v = d.alpha * acc[r][c];
        if (d.beta != 0.0) v = fma(d.beta, d.C[gi + (int64_t)gj * d.ldc], v);
        d.C[gi + (int64_t)gj * d.ldc] = v;
        if (d.C2) d.C2[gj + (int64_t)gi * d.ldc2] = v;
      }
    }
}

// ---------------------------------------------------------------------------
// Early-stopping column-pivoted Householder QR, one interface per workgroup.
// ---------------------------------------------------------------------------
constexpr int kCpqrThreads = 256;

__global__ __launch_bounds__(kCpqrThreads) void k_cpqr(const CpqrDesc* descs, const CpqrNbr* nbrs,
                                                        int32_t* n_cur, int32_t* out_r,
                                                        int32_t* out_r2, int32_t* out_k,
                                                        double eps, double eps_stop, int32_t max_k) {
  extern __shared__ double sm[];
  __shared__ double red[kCpqrThreads / kWave];
  __shared__ int ired[kCpqrThreads / kWave];
  const CpqrDesc d = descs[blockIdx.x];
  const int a = d.a;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  constexpr int NW = kCpqrThreads / kWave;
  double* nrm2 = sm;
  double* v = sm + max_k;
  double* Y = d.Y;

  // gather W = [B_{p,w1} ... B_{p,wm}] with the neighbours' current widths
  int k = 0;
  for (int64_t e = d.nb0; e < d.nb1; ++e) {
    const CpqrNbr nb = nbrs[e];
    const int wc = n_cur[nb.w];
    const double* src = d.panel + nb.col * a;
    double* dst = Y + (int64_t)k * a;
    for (int64_t idx = tid; idx < (int64_t)a * wc; idx += kCpqrThreads) dst[idx] = src[idx];
    k += wc;
  }
  __syncthreads();
  for (int c = wid; c < k; c += NW) {
    double s = 0.0;
    for (int i = lane; i < a; i += kWave) {
      const double y = Y[i + (int64_t)c * a];
      s = fma(y, y, s);
    }
    s = wave_sum(s);
    if (lane == 0) nrm2[c] = s;
  }
  __syncthreads();

  int r = -1;
  int j = 0;
  double R00 = 0.0;
  const int jmax = min(a, k);
  for (; j < jmax; ++j) {
    double m = -1.0;
    for (int c = tid; c < k; c += kCpqrThreads) m = fmax(m, nrm2[c]);
    m = block_max<kCpqrThreads>(m, red);
    if (m < 0.0) break;
    const double thr = m * (1.0 - kPivotTieRtol);
    int cand = INT_MAX;
    for (int c = tid; c < k; c += kCpqrThreads)
      if (nrm2[c] >= 0.0 && nrm2[c] >= thr) { cand = c; break; }
    cand = block_min_int<kCpqrThreads>(cand, ired);
    double s = 0.0;
    for (int i = j + tid; i < a; i += kCpqrThreads) {
      const double y = Y[i + (int64_t)cand * a];
      s = fma(y, y, s);
    }
    s = block_sum<kCpqrThreads>(s, red);
    const double nrm = sqrt(s);
    if (j == 0) R00 = nrm;
    if (nrm == 0.0 || nrm < eps_stop * R00) break;
    if (r < 0 && nrm < eps * R00) r = j;
    const double alpha = Y[j + (int64_t)cand * a];
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double denom = alpha - beta;
    const double tau = (beta - alpha) / beta;
    for (int i = j + tid; i < a; i += kCpqrThreads) {
      const double vi = i == j ? 1.0 : Y[i + (int64_t)cand * a] / denom;
      v[i] = vi;
      d.V[i + (int64_t)j * a] = vi;
    }
    if (tid == 0) d.tau[j] = tau;
    __syncthreads();
    for (int c = wid; c < k; c += NW) {
      if (c == cand || nrm2[c] < 0.0) continue;
      double* col = Y + (int64_t)c * a;
      double w = 0.0;
      for (int i = j + lane; i < a; i += kWave) w = fma(v[i], col[i], w);
      w = wave_sum(w) * tau;
      double s2 = 0.0;
      for (int i = j + lane; i < a; i += kWave) {
        const double y = fma(-w, v[i], col[i]);
        col[i] = y;
        if (i > j) s2 = fma(y, y, s2);
      }
      s2 = wave_sum(s2);
      if (lane == 0) nrm2[c] = s2;
    }
    for (int i = j + tid; i < a; i += kCpqrThreads) Y[i + (int64_t)cand * a] = i == j ? beta : 0.0;
    __syncthreads();
    if (tid == 0) nrm2[cand] = -1.0;
    __syncthreads();
  }
  const int nref = j;
  if (r < 0) r = nref;

  // coarse rows back into p's panel and, transposed, into the neighbours' panels
  int kk = 0;
  for (int64_t e = d.nb0; e < d.nb1; ++e) {
    const CpqrNbr nb = nbrs[e];
    const int wc = n_cur[nb.w];
    for (int idx = tid; idx < r * wc; idx += kCpqrThreads) {
      const int i = idx % r, c = idx / r;
      const double y = Y[i + (int64_t)(kk + c) * a];
      d.panel[i + (nb.col + c) * a] = y;
      nb.blk_wp[c + (int64_t)i * nb.ldw] = y;
    }
    kk += wc;
  }
  for (int idx = tid; idx < r * r; idx += kCpqrThreads) {
    const int i = idx % r, c = idx / r;
    d.panel[i + (d.diag_col + c) * a] = i == c ? 1.0 : 0.0;
  }
  if (tid == 0) {
    out_k[d.p] = k;
    out_r[d.p] = r;
    out_r2[d.p] = nref;
  }
  __syncthreads();
  if (tid == 0) n_cur[d.p] = r;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_scatter(const double* vals, const int64_t* dest, int64_t nnz, double* panels) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    panels[dest[e]] = vals[e];
}

__global__ __launch_bounds__(256) void k_copy(const CopyDesc* descs) {
  const CopyDesc d = descs[blockIdx.x];
  for (int64_t idx = threadIdx.x; idx < (int64_t)d.m * d.n; idx += blockDim.x) {
    const int i = (int)(idx % d.m), j = (int)(idx / d.m);
    d.dst[i + (int64_t)j * d.ldd] = d.src[i + (int64_t)j * d.lds];
  }
}

inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

void launch_scatter(const double* vals, const int64_t* dest, int64_t nnz, double* panels,
                    hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(nnz, 256)), dim3(256), 0, s, vals, dest, nnz, panels);
}

void launch_potrf_inv(const PotrfDesc* d, int32_t count, int32_t max_n, int32_t* info,
                      hipStream_t s) {
  if (count <= 0) return;
  const int nl = max_n <= kPotrfLdsMax ? max_n : kPotrfLdsMax;
  size_t lds = (size_t)nl * nl * sizeof(double) + (size_t)max_n * sizeof(double);
  hipLaunchKernelGGL(k_potrf_inv, dim3(count), dim3(kPotrfThreads), lds, s, d, info);
}

void launch_gemm(const GemmDesc* d, const GemmTerm* t, const TileRef* tiles, int64_t ntiles,
                 hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gemm, dim3((unsigned)ntiles), dim3(kGemmThreads), 0, s, d, t, tiles);
}

void launch_cpqr(const CpqrDesc* d, const CpqrNbr* nb, int32_t count, int32_t* n_cur,
                 int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps, double eps_stop,
                 int32_t max_a, int32_t max_k, hipStream_t s) {
  if (count <= 0) return;
  size_t lds = ((size_t)max_k + max_a) * sizeof(double);
  hipLaunchKernelGGL(k_cpqr, dim3(count), dim3(kCpqrThreads), lds, s, d, nb, n_cur, out_r, out_r2,
                     out_k, eps, eps_stop, max_k);
}

void launch_copy(const CopyDesc* d, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)count), dim3(256), 0, s, d);
}

}  // namespace spand
