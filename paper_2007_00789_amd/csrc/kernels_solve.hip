// HIP kernels of the preconditioner apply and of PCG.  Vectors, scratch and
// accumulation are FP64; the factor entries the apply reads are of the
// factor's element type (the kernels are templates on it, MT: double or float).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "apply.h"

namespace spand {

namespace {

constexpr int kWave = 64;
constexpr int kT = 256;
constexpr int kST = 512;   // threads of the E-tile kernels
// right-hand sides per pass of the interior GEMVs (bounds their LDS partial sums)
__host__ __device__ constexpr int ap_rb(int nrhs) { return nrhs > 4 ? 2 : 4; }

// DPP move of a double (two 32-bit halves); lanes whose source is invalid read 0.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes (all active), returned to every lane: quad
// permutations and row rotations reduce each row of 16 lanes, row broadcasts
// 15 and 31 carry the row sums so that lane 63 holds the total.
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

// all threads get the block sum; `red` holds kT/64 doubles
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kT / kWave; ++w) s += red[w];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Workgroup building blocks.  Matrices are column-major in global memory;
// vectors of the cluster being processed are staged in LDS (rows x nrhs).
// ---------------------------------------------------------------------------
constexpr int kNW = kT / kWave;
constexpr int kBatch = 8;   // columns per wave iteration (independent loads in flight)
constexpr int kChunk = 1024;  // staged neighbour values of the backward E product

// acc_out[i + r*rows] = sum_{c<cols} M[i + c*ld] z[pos[c] + r*ldz] for i < rows.
// The gathered values are staged in LDS (chunks of kChunk columns, all
// threads loading); then lanes hold rows and waves split the columns, and the
// per-wave partial sums are reduced in a fixed order.
// stage: LDS of kChunk * nrhs, part: LDS of kNW * rows * nrhs.  Ends with a barrier.
template <class MT>
__device__ void wg_rowsum_gather(const MT* __restrict__ M, int64_t ld, int rows, int cols,
                                 const int32_t* __restrict__ pos, const double* __restrict__ z,
                                 int64_t ldz, int nrhs, double* __restrict__ stage,
                                 double* __restrict__ part, double* __restrict__ acc_out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int idx = threadIdx.x; idx < kNW * rows * nrhs; idx += kT) part[idx] = 0.0;
  for (int c0 = 0; c0 < cols; c0 += kChunk) {
    const int cn = min(kChunk, cols - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < cn * nrhs; idx += kT) {
      const int c = idx % cn, r = idx / cn;
      stage[idx] = z[pos[c0 + c] + r * ldz];
    }
    __syncthreads();
    for (int i0 = 0; i0 < rows; i0 += kWave) {
      const int i = i0 + lane;
      if (i >= rows) continue;
      for (int r = 0; r < nrhs; ++r) {
        double acc = 0.0;
#pragma unroll 8
        for (int c = wid; c < cn; c += kNW) acc = fma(M[i + (int64_t)(c0 + c) * ld], stage[c + r * cn], acc);
        part[(wid * nrhs + r) * rows + i] += acc;
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < rows * nrhs; idx += kT) {
    const int i = idx % rows, r = idx / rows;
    double sacc = 0.0;
#pragma unroll
    for (int w = 0; w < kNW; ++w) sacc += part[(w * nrhs + r) * rows + i];
    acc_out[idx] = sacc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Helpers for NT-thread workgroups.
// ---------------------------------------------------------------------------
// The GEMV helpers below keep many loads in flight per lane: a lane loads
// every 64-row chunk it needs (RC chunks, 64*RC rows per block) for a small
// batch of columns before the first FMA, so a workgroup's product costs a few
// memory round trips instead of one per chunk.  The interior and scaling
// kernels come in two shapes: CB = 8 columns per wave batch (few large
// workgroups: fewer round trips) and CB = 2 (many small workgroups: 76 VGPRs
// instead of 248, so four times the waves per SIMD).
constexpr int kApWide = 8, kApNarrow = 2;
// launches of at least this many workgroups take the narrow shape
constexpr int kApNarrowFrom = 512;
// out[c + r*ldo] = sum_{i<rows} M[i + c*ld] x[i + r*ldx]: one wave per batch of
// CB columns, lanes over rows (coalesced, RC chunks of 64 per block), one wave
// reduction per output.
template <int NT, int RC, int CB, class MT>
__device__ void wgt_coldots(const MT* __restrict__ M, int64_t ld, int rows, int cols,
                            const double* __restrict__ x, int ldx, int nrhs, double* __restrict__ out,
                            int64_t ldo) {
  constexpr int NW = NT / kWave, kRC = RC;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int c0 = wid * CB; c0 < cols; c0 += NW * CB) {
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
      double acc[CB][4];
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[q][rr] = 0.0;
      for (int ib = 0; ib < rows; ib += kWave * kRC) {
        double m[kRC][CB];
#pragma unroll
        for (int t = 0; t < kRC; ++t)
#pragma unroll
          for (int q = 0; q < CB; ++q) {
            const int i = ib + lane + kWave * t;
            m[t][q] = (i < rows && c0 + q < cols) ? M[i + (int64_t)(c0 + q) * ld] : 0.0;
          }
#pragma unroll
        for (int t = 0; t < kRC; ++t) {
          const int i = ib + lane + kWave * t;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const double xv = (i < rows && r0 + rr < nrhs) ? x[i + (r0 + rr) * ldx] : 0.0;
#pragma unroll
            for (int q = 0; q < CB; ++q) acc[q][rr] = fma(m[t][q], xv, acc[q][rr]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          if (r0 + rr >= nrhs) break;
          const double v = wave_sum(acc[q][rr]);
          if (lane == 0 && c0 + q < cols) out[c0 + q + (int64_t)(r0 + rr) * ldo] = v;
        }
    }
  }
}

// y[i + r*ldy] += sign * sum_{c<cols} M[i + c*ld] w[c + r*ldw] for i < rows:
// lanes over rows (coalesced, RC chunks of 64 per lane), waves over columns
// (CU columns in flight), rb right-hand sides per pass; per-wave partial sums
// in LDS (part: NW x rows x rb) added in wave order.  Ends with a barrier.
template <int NT, int RC, int CU, class MT>
__device__ void wgt_gemv_acc(const MT* __restrict__ M, int64_t ld, int rows, int cols,
                             const double* __restrict__ w, int ldw, int nrhs, double sign,
                             double* __restrict__ y, int ldy, double* __restrict__ part, int rb) {
  constexpr int NW = NT / kWave, kRC = RC;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int r0 = 0; r0 < nrhs; r0 += rb) {
    const int nr = min(rb, nrhs - r0);
    for (int ib = 0; ib < rows; ib += kWave * kRC) {
      double acc[kRC][4];
#pragma unroll
      for (int t = 0; t < kRC; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[t][rr] = 0.0;
#pragma unroll CU
      for (int c = wid; c < cols; c += NW) {
        double wv[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) wv[rr] = rr < nr ? w[c + (r0 + rr) * ldw] : 0.0;
#pragma unroll
        for (int t = 0; t < kRC; ++t) {
          const int i = ib + lane + kWave * t;
          const double m = i < rows ? M[i + (int64_t)c * ld] : 0.0;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) acc[t][rr] = fma(m, wv[rr], acc[t][rr]);
        }
      }
#pragma unroll
      for (int t = 0; t < kRC; ++t) {
        const int i = ib + lane + kWave * t;
        if (i < rows)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            if (rr < nr) part[(wid * rows + i) * rb + rr] = acc[t][rr];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * nr; idx += NT) {
      const int i = idx / nr, rr = idx - i * nr;
      double sacc = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) sacc += part[(q * rows + i) * rb + rr];
      y[i + (r0 + rr) * ldy] += sign * sacc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// forward interior: z_s <- L^{-1} z_s ; t = G^T z_s
// ---------------------------------------------------------------------------
template <class MT, int CB>
__global__ __launch_bounds__(kT) void k_ap_int_fwd(const ApInt* descs, double* z, int64_t ldz,
                                                   int nrhs, double* T) {
  extern __shared__ double sm[];
  const ApInt d = descs[blockIdx.x];
  const int n = d.n, k = d.k;
  double* xs = sm;             // n x nrhs
  double* ys = sm + n * nrhs;  // n x nrhs
  double* part = ys + n * nrhs;   // kNW x n x ap_rb(nrhs)
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    xs[idx] = z[d.pos[i] + r * ldz];
    ys[idx] = 0.0;
  }
  __syncthreads();
  // ys = L^{-1} xs (L^{-1} is stored with zeros above its diagonal)
  wgt_gemv_acc<kT, 1, CB>(static_cast<const MT*>(d.Linv), n, n, n, xs, n, nrhs, 1.0, ys, n, part,
                          ap_rb(nrhs));
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    z[d.pos[i] + r * ldz] = ys[idx];
  }
  if (k == 0) return;
  wgt_coldots<kT, 1, CB>(static_cast<const MT*>(d.G), n, n, k, ys, n, nrhs, T + d.toff * nrhs, k);
}

// ---------------------------------------------------------------------------
// gather: z_w -= sum of slices; optional scaling z_w <- Zinv z_w
// ---------------------------------------------------------------------------
template <class MT>
__global__ __launch_bounds__(kT) void k_ap_gather(const ApGat* descs, const ApSrc* src, double* z,
                                                  int64_t ldz, int nrhs, const double* T,
                                                  double* Y) {
  extern __shared__ double sm[];
  const ApGat d = descs[blockIdx.x];
  const int n = d.n;
  double* xs = sm;
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = z[d.pos[i] + r * ldz];
    for (int64_t e = d.src0; e < d.src1; ++e) {
      const ApSrc sv = src[e];
      acc -= T[sv.toff * nrhs + sv.col + i + (int64_t)r * sv.ld];
    }
    if (d.split) Y[d.yoff * nrhs + idx] = acc;
    else if (!d.Zinv) z[d.pos[i] + r * ldz] = acc;
    else xs[idx] = acc;
  }
  if (!d.Zinv || d.split) return;
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = 0.0;
#pragma unroll 8
    for (int m = 0; m <= i; ++m)
      acc = fma((double)static_cast<const MT*>(d.Zinv)[i + (int64_t)m * n], xs[m + r * n], acc);
    z[d.pos[i] + r * ldz] = acc;
  }
}

// ---------------------------------------------------------------------------
// E tiles.  Forward: t[c] = sum_i E[i, c] z_f[i] over a tile of kEtTileF
// columns: lanes over the columns (rows of E^T are contiguous), the waves split
// the rows, and the per-wave partial sums are added in wave order.
// LDS: z_f (nf x nrhs) | part (kSNW x 64 x 4).
// ---------------------------------------------------------------------------
template <class MT>
__global__ __launch_bounds__(kST) void k_ap_et_fwd(const ApEt* descs, const double* z, int64_t ldz,
                                                   int nrhs, double* T) {
  extern __shared__ double sm[];
  constexpr int NW = kST / kWave;
  const ApEt d = descs[blockIdx.x];
  const int nf = d.nf, lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double* zf = sm;
  double* part = sm + nf * nrhs;
  for (int idx = threadIdx.x; idx < nf * nrhs; idx += kST) {
    const int i = idx % nf, r = idx / nf;
    zf[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  const int per = (nf + NW - 1) / NW, i0 = min(nf, wid * per), i1 = min(nf, i0 + per);
  const bool col = lane < d.cn;
  const MT* e = static_cast<const MT*>(d.Et) + d.c0 + (col ? lane : 0);
  double* t = T + d.off * nrhs + d.c0 + lane;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (col) {
#pragma unroll 8
      for (int i = i0; i < i1; ++i) {
        const double ev = e[(int64_t)i * d.lde];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          if (r0 + rr < nrhs) acc[rr] = fma(ev, zf[i + (r0 + rr) * nf], acc[rr]);
      }
    }
    // partial sums by column of the right-hand side: consecutive lanes write
    // consecutive doubles (no LDS bank conflicts)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) part[rr * kST + wid * kWave + lane] = acc[rr];
    __syncthreads();
    if (wid == 0 && col)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        if (r0 + rr >= nrhs) break;
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sacc += part[rr * kST + q * kWave + lane];
        t[(int64_t)(r0 + rr) * d.k] = sacc;
      }
    __syncthreads();
  }
}

// Backward: part[i] = sum_{c in tile} E[i, c] y_W[c] for every fine row i.
// The tile's neighbour values are staged in LDS (cn x nrhs); each wave takes
// four rows of E at a time with all of the tile's columns in flight (lanes over
// columns, up to kEtTileB / 64 chunks per lane).
template <class MT>
__global__ __launch_bounds__(kST) void k_ap_et_bwd(const ApEt* descs, const double* z, int64_t ldz,
                                                   int nrhs, double* P) {
  extern __shared__ double sm[];
  constexpr int NW = kST / kWave, CH = kEtTileB / kWave;
  const ApEt d = descs[blockIdx.x];
  const int nf = d.nf, cn = d.cn;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double* yw = sm;
  for (int idx = threadIdx.x; idx < cn * nrhs; idx += kST) {
    const int c = idx % cn, r = idx / cn;
    yw[idx] = z[d.pos[d.c0 + c] + r * ldz];
  }
  __syncthreads();
  double* out = P + d.off * nrhs;
  for (int i0 = wid * 4; i0 < nf; i0 += NW * 4) {
    double ev[4][CH];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int c = lane + kWave * t;
        ev[q][t] = (i0 + q < nf && c < cn)
                       ? (double)static_cast<const MT*>(d.Et)[d.c0 + c + (int64_t)(i0 + q) * d.lde]
                       : 0.0;
      }
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
      double acc[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[q][rr] = 0.0;
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int c = lane + kWave * t;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const double yv = (c < cn && r0 + rr < nrhs) ? yw[c + (r0 + rr) * cn] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q][rr] = fma(ev[q][t], yv, acc[q][rr]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          if (r0 + rr >= nrhs) break;
          const double v = wave_sum(acc[q][rr]);
          if (lane == 0 && i0 + q < nf) out[i0 + q + (int64_t)(r0 + rr) * nf] = v;
        }
    }
  }
}

// ---------------------------------------------------------------------------
// wide WY apply (one colour): Q^T x = x - V ((VT)^T x) forward, Q y = y - VT
// (V^T y) backward, each as a dots launch and an update launch spread over
// column blocks and row blocks of every interface of the colour.
// ---------------------------------------------------------------------------
// x_i of interface row i: z at its position, minus (backward) the E tiles'
// partial sums for the fine rows, added in tile order
__device__ __forceinline__ double wy_in(const ApSp& d, const double* __restrict__ z, int64_t ldz,
                                        const double* __restrict__ P, int i, int r, int nrhs) {
  double v = z[d.pos[i] + (int64_t)r * ldz];
  if (P && i >= d.f0 && i < d.f1) {
    const int nf = d.f1 - d.f0;
    for (int t = 0; t < d.ntiles; ++t)
      v -= P[(d.part0 + (int64_t)t * nf) * nrhs + (i - d.f0) + (int64_t)r * nf];
  }
  return v;
}

// u[j0 + c] = sum_i M[i, j0 + c] x_i for kApWyCB columns: threads over rows
// (columns of M are contiguous), two rows per thread in flight, wave sums,
// then the waves in order.
template <class MT>
__global__ __launch_bounds__(kApWyThreads) void k_ap_wy_dots(const ApWyTask* tasks, const ApSp* descs,
                                                            const double* __restrict__ z, int64_t ldz,
                                                            int nrhs, const double* __restrict__ P,
                                                            double* __restrict__ U, int64_t usz,
                                                            int fwd) {
  constexpr int NW = kApWyThreads / kWave, CB = kApWyCB;
  __shared__ double red[NW][CB * 4];
  const ApWyTask tk = tasks[blockIdx.x];
  const ApSp d = descs[tk.sp];
  const MT* __restrict__ M = static_cast<const MT*>(fwd ? d.VT : d.V);
  const int a = d.a, j0 = tk.i0, cn = min(CB, d.nref - j0);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const double* Pp = fwd ? nullptr : P;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    double acc[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[c][rr] = 0.0;
    for (int i0 = threadIdx.x; i0 < a; i0 += 2 * kApWyThreads) {
      double x[2][4], m[2][CB];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = i0 + t * kApWyThreads;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          x[t][rr] = (i < a && r0 + rr < nrhs) ? wy_in(d, z, ldz, Pp, i, r0 + rr, nrhs) : 0.0;
#pragma unroll
        for (int c = 0; c < CB; ++c) m[t][c] = (i < a && c < cn) ? M[i + (int64_t)(j0 + c) * a] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) acc[c][rr] = fma(m[t][c], x[t][rr], acc[c][rr]);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        if (r0 + rr >= nrhs) break;   // no reduction for the padding columns
        const double v = wave_sum(acc[c][rr]);
        if (lane == 0) red[wid][c * 4 + rr] = v;
      }
    __syncthreads();
    if (threadIdx.x < CB * 4) {
      const int c = threadIdx.x / 4, rr = threadIdx.x % 4;
      if (c < cn && r0 + rr < nrhs) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) v += red[q][c * 4 + rr];
        U[d.uoff + j0 + c + (int64_t)(r0 + rr) * usz] = v;
      }
    }
    __syncthreads();
  }
}

// x_i -= sum_j N[i, j] u_j for kApWyRB rows: 16 rows x 16 column groups (a
// wave reads 4 x 16 consecutive rows of 4 columns), eight columns per thread
// in flight, u staged in LDS in chunks, the groups summed in order.
constexpr int kApWyUChunk = 512;
template <class MT>
__global__ __launch_bounds__(kApWyThreads) void k_ap_wy_update(const ApWyTask* tasks,
                                                            const ApSp* descs, double* z,
                                                            int64_t ldz, int nrhs,
                                                            const double* __restrict__ P,
                                                            const double* __restrict__ U,
                                                            int64_t usz, int fwd) {
  constexpr int RB = kApWyRB, NG = kApWyThreads / RB, UC = kApWyUChunk;
  __shared__ double red[NG][RB * 4];
  __shared__ double us[UC * 4];
  const ApWyTask tk = tasks[blockIdx.x];
  const ApSp d = descs[tk.sp];
  const MT* __restrict__ N = static_cast<const MT*>(fwd ? d.V : d.VT);
  const int a = d.a, nref = d.nref;
  const int rl = threadIdx.x % RB, g = threadIdx.x / RB;
  const int i = tk.i0 + rl;
  const double* u = U + d.uoff;
  const double* Pp = fwd ? nullptr : P;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = min(4, nrhs - r0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int jc = 0; jc < nref; jc += UC) {
      const int jn = min(UC, nref - jc);
      __syncthreads();
      for (int idx = threadIdx.x; idx < jn * 4; idx += kApWyThreads) {
        const int jj = idx / 4, rr = idx % 4;
        us[idx] = rr < nr ? u[jc + jj + (int64_t)(r0 + rr) * usz] : 0.0;
      }
      __syncthreads();
      if (i < a) {
        for (int j = g; j < jn; j += NG * 8) {
          double nv[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int jj = j + t * NG;
            nv[t] = jj < jn ? N[i + (int64_t)(jc + jj) * a] : 0.0;
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int jj = min(j + t * NG, jn - 1);   // nv[t] is 0 past the end
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) acc[rr] = fma(nv[t], us[jj * 4 + rr], acc[rr]);
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) red[g][rl * 4 + rr] = acc[rr];
    __syncthreads();
    if (threadIdx.x < RB * 4) {
      const int r2 = threadIdx.x / 4, rr = threadIdx.x % 4, i2 = tk.i0 + r2;
      if (i2 < a && rr < nr) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) v += red[q][r2 * 4 + rr];
        z[d.pos[i2] + (int64_t)(r0 + rr) * ldz] = wy_in(d, z, ldz, Pp, i2, r0 + rr, nrhs) - v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// split GEMV (large interiors): rows and column-dot kernels over ApMv tasks
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mv_x(const ApMv& d, const double* __restrict__ z, int64_t ldz,
                                       const double* __restrict__ S, int nrhs, int j, int r) {
  return d.xpos ? z[d.xpos[j] + (int64_t)r * ldz] : S[d.xoff * nrhs + j + (int64_t)r * d.xld];
}

// kApMvRB rows per task: 16 rows x 16 column groups, x staged in LDS in
// chunks, eight columns per thread in flight, groups summed in order.
constexpr int kApMvChunk = 512;
template <class MT>
__global__ __launch_bounds__(kApWyThreads) void k_ap_mv_rows(const ApMvTask* tasks, const ApMv* descs,
                                                            double* z, int64_t ldz, int nrhs,
                                                            const double* __restrict__ S,
                                                            double* __restrict__ O) {
  constexpr int RB = kApMvRB, NG = kApWyThreads / RB, UC = kApMvChunk;
  __shared__ double red[NG][RB * 4];
  __shared__ double xs[UC * 4];
  const ApMvTask tk = tasks[blockIdx.x];
  const ApMv d = descs[tk.mv];
  const int rl = threadIdx.x % RB, g = threadIdx.x / RB;
  const int i = tk.i0 + rl;
  const int jmax = d.tri ? min(d.cols, tk.i0 + RB) : d.cols;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = min(4, nrhs - r0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int jc = 0; jc < jmax; jc += UC) {
      const int jn = min(UC, jmax - jc);
      __syncthreads();
      for (int idx = threadIdx.x; idx < jn * 4; idx += kApWyThreads) {
        const int jj = idx / 4, rr = idx % 4;
        xs[idx] = rr < nr ? mv_x(d, z, ldz, S, nrhs, jc + jj, r0 + rr) : 0.0;
      }
      __syncthreads();
      if (i < d.rows) {
        for (int j = g; j < jn; j += NG * 8) {
          double mv[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int jj = j + t * NG;
            mv[t] = jj < jn ? (double)static_cast<const MT*>(d.M)[i + (int64_t)(jc + jj) * d.ld] : 0.0;
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int jj = min(j + t * NG, jn - 1);   // mv[t] is 0 past the end
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) acc[rr] = fma(mv[t], xs[jj * 4 + rr], acc[rr]);
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) red[g][rl * 4 + rr] = acc[rr];
    __syncthreads();
    if (threadIdx.x < RB * 4) {
      const int r2 = threadIdx.x / 4, rr = threadIdx.x % 4, i2 = tk.i0 + r2;
      if (i2 < d.rows && rr < nr) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) v += red[q][r2 * 4 + rr];
        if (d.bpos) v = z[d.bpos[i2] + (int64_t)(r0 + rr) * ldz] - v;
        if (d.opos) z[d.opos[i2] + (int64_t)(r0 + rr) * ldz] = v;
        else O[d.ooff * nrhs + i2 + (int64_t)(r0 + rr) * d.old] = v;
      }
    }
    __syncthreads();
  }
}

// 4 x kApMvCB columns per task, one wave per kApMvCB columns: lanes over rows
// (columns of M are contiguous), two rows per lane in flight, one wave sum per
// output.
template <class MT>
__global__ __launch_bounds__(kApWyThreads) void k_ap_mv_cols(const ApMvTask* tasks, const ApMv* descs,
                                                            double* z, int64_t ldz, int nrhs,
                                                            const double* __restrict__ S,
                                                            double* __restrict__ O) {
  constexpr int CB = kApMvCB;
  const ApMvTask tk = tasks[blockIdx.x];
  const ApMv d = descs[tk.mv];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (d.wpos && tk.i0 == 0)
    for (int idx = threadIdx.x; idx < d.rows * nrhs; idx += kApWyThreads) {
      const int i = idx % d.rows, r = idx / d.rows;
      z[d.wpos[i] + (int64_t)r * ldz] = mv_x(d, z, ldz, S, nrhs, i, r);
    }
  const int c0 = tk.i0 + wid * CB, cn = min(CB, d.cols - c0);
  if (cn <= 0) return;
  const int i_lo = d.tri ? c0 : 0;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    double acc[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[c][rr] = 0.0;
    for (int ib = i_lo + lane; ib < d.rows; ib += 2 * kWave) {
      double x[2][4], m[2][CB];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = ib + t * kWave;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          x[t][rr] = (i < d.rows && r0 + rr < nrhs) ? mv_x(d, z, ldz, S, nrhs, i, r0 + rr) : 0.0;
#pragma unroll
        for (int c = 0; c < CB; ++c)
          m[t][c] = (i < d.rows && c < cn) ? (double)static_cast<const MT*>(d.M)[i + (int64_t)(c0 + c) * d.ld] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) acc[c][rr] = fma(m[t][c], x[t][rr], acc[c][rr]);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        if (r0 + rr >= nrhs) break;   // no reduction for the padding columns
        const double v = wave_sum(acc[c][rr]);
        if (lane == 0 && c < cn) {
          if (d.opos) z[d.opos[c0 + c] + (int64_t)(r0 + rr) * ldz] = v;
          else O[d.ooff * nrhs + c0 + c + (int64_t)(r0 + rr) * d.old] = v;
        }
      }
  }
}

// backward scaling: y_w <- Zinv^T y_w (column dots of Zinv)
template <class MT, int CB>
__global__ __launch_bounds__(kT) void k_ap_scale_bwd(const ApScale* descs, double* z, int64_t ldz,
                                                     int nrhs) {
  extern __shared__ double sm[];
  const ApScale d = descs[blockIdx.x];
  const int n = d.n;
  double* xs = sm;
  double* ys = sm + n * nrhs;
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    xs[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  wgt_coldots<kT, 1, CB>(static_cast<const MT*>(d.Zinv), n, n, n, xs, n, nrhs, ys, n);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    z[d.pos[i] + r * ldz] = ys[idx];
  }
}

// backward interior: y_s <- L^{-T} (y_s - G y_W)
// LDS: us (n x nrhs) | ys (n x nrhs) | part (kNW x n x nrhs) | stage (kChunk x nrhs)
template <class MT, int CB>
__global__ __launch_bounds__(kT) void k_ap_int_bwd(const ApInt* descs, double* z, int64_t ldz,
                                                   int nrhs) {
  extern __shared__ double sm[];
  const ApInt d = descs[blockIdx.x];
  const int n = d.n, k = d.k;
  double* us = sm;
  double* ys = sm + n * nrhs;
  double* part = ys + n * nrhs;
  double* stage = part + kNW * n * nrhs;
  if (k > 0)
    wg_rowsum_gather(static_cast<const MT*>(d.G), n, n, k, d.nbr_pos, z, ldz, nrhs, stage, part, ys);
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    us[idx] = z[d.pos[i] + r * ldz] - (k > 0 ? ys[idx] : 0.0);
  }
  __syncthreads();
  wgt_coldots<kT, 1, CB>(static_cast<const MT*>(d.Linv), n, n, n, us, n, nrhs, ys, n);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    z[d.pos[i] + r * ldz] = ys[idx];
  }
}

// ---------------------------------------------------------------------------
// PCG helpers
// ---------------------------------------------------------------------------
__global__ void k_spmv(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                       int nrhs, const double* x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    for (int r = 0; r < nrhs; ++r) {
      double acc = 0.0;
      for (int64_t q = b; q < e; ++q) acc = fma(vals[q], x[colind[q] + r * n], acc);
      y[i + r * n] = acc;
    }
  }
}

// block (b, s, c) sums its chunk of segment s, column c
__global__ __launch_bounds__(kT) void k_dot_partial(const double* x, const double* y, int64_t n,
                                                    const int64_t* seg_off, double* partial) {
  __shared__ double red[kT / kWave];
  const int b = blockIdx.x, sg = blockIdx.y, c = blockIdx.z, bps = gridDim.x;
  const int nrhs = gridDim.z;
  const double* xr = x + (int64_t)c * n;
  const double* yr = y + (int64_t)c * n;
  const int64_t o0 = seg_off[sg], o1 = seg_off[sg + 1];
  const int64_t chunk = (o1 - o0 + bps - 1) / bps;
  const int64_t lo = o0 + (int64_t)b * chunk, hi = min(o1, lo + chunk);
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kT) acc = fma(xr[i], yr[i], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[((int64_t)sg * nrhs + c) * bps + b] = acc;
}

// one wave per (segment, column): lanes over the partial sums, one wave sum
__global__ __launch_bounds__(kWave) void k_dot_final(const double* partial, int bps, int count,
                                                     double* out) {
  const int e = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < bps; i += kWave) s += partial[(int64_t)e * bps + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[e] = s;
}

__global__ void k_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rho,
                         const double* pq, const int32_t* active, const int32_t* seg_id, int64_t n,
                         int nrhs) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * nrhs;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n);
    const int e = (seg_id ? seg_id[idx - (int64_t)c * n] : 0) * nrhs + c;
    if (!active[e]) continue;
    const double alpha = rho[e] / pq[e];
    x[idx] = fma(alpha, p[idx], x[idx]);
    r[idx] = fma(-alpha, q[idx], r[idx]);
  }
}

__global__ void k_pcg_p(double* p, const double* z, const double* rho, const double* rho_new,
                        const int32_t* active, const int32_t* seg_id, int64_t n, int nrhs,
                        int first) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * nrhs;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n);
    const int e = (seg_id ? seg_id[idx - (int64_t)c * n] : 0) * nrhs + c;
    if (!active[e]) continue;
    p[idx] = first ? z[idx] : fma(rho_new[e] / rho[e], p[idx], z[idx]);
  }
}

__global__ void k_copy_rho(double* rho, const double* rho_new, const int32_t* active, int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count && active[e]) rho[e] = rho_new[e];
}

__global__ void k_residual(const double* b, double* y, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b[i] - y[i];
}

__global__ void k_copy_vec(const double* s, double* d, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// prescale: d_i = 1 / sqrt(a_ii) per row (the lowest row with a_ii <= 0, or
// no diagonal entry, into *bad), then every value a_ij (d_i d_j), which keeps
// the scaled values exactly symmetric
__global__ void k_prescale_diag(const int64_t* rowptr, const int32_t* colind, const double* vals,
                                int64_t n, double* d, int32_t* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (colind[e] == i) a += vals[e];
    if (a > 0.0) d[i] = 1.0 / sqrt(a);
    else {
      d[i] = 0.0;
      atomicMin(bad, (int32_t)i);
    }
  }
}

__global__ void k_prescale_vals(const int64_t* rowptr, const int32_t* colind, const double* vals,
                                int64_t n, const double* d, double* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double di = d[i];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) out[e] = vals[e] * (di * d[colind[e]]);
  }
}

// y = d o x for nrhs columns of n (x and y may alias)
__global__ void k_scale_vec(const double* x, const double* d, double* y, int64_t n, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = d[i % n] * x[i];
}

__global__ void k_fill_i32(int32_t* p, int32_t v) { *p = v; }

inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 16384) g = 16384;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

// the factor's element type selects the kernel instance
#define SPAND_AP_LAUNCH(f32, K, grid, block, lds, s, ...)                         \
  do {                                                                          \
    if (f32) hipLaunchKernelGGL(K<float>, grid, block, lds, s, __VA_ARGS__);     \
    else hipLaunchKernelGGL(K<double>, grid, block, lds, s, __VA_ARGS__);        \
  } while (0)

void launch_ap_int_fwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       double* T, int32_t max_n, bool f32, hipStream_t s) {
  if (count <= 0) return;
  const size_t lds = ((size_t)2 * max_n * nrhs + (size_t)kNW * max_n * ap_rb(nrhs)) * sizeof(double);
  if (count >= kApNarrowFrom) {
    if (f32) hipLaunchKernelGGL((k_ap_int_fwd<float, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs, T);
    else hipLaunchKernelGGL((k_ap_int_fwd<double, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs, T);
  } else {
    if (f32) hipLaunchKernelGGL((k_ap_int_fwd<float, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs, T);
    else hipLaunchKernelGGL((k_ap_int_fwd<double, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs, T);
  }
}
void launch_ap_gather(const ApGat* d, const ApSrc* src, int32_t count, double* z, int64_t ldz,
                      int32_t nrhs, const double* T, int32_t max_n, bool f32, hipStream_t s,
                      double* Y) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_gather, dim3(count), dim3(kT), (size_t)max_n * nrhs * sizeof(double), s,
                  d, src, z, ldz, nrhs, T, Y);
}
void launch_ap_et_fwd(const ApEt* d, int32_t count, const double* z, int64_t ldz, int32_t nrhs,
                      double* T, int32_t max_nf, bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_et_fwd, dim3(count), dim3(kST),
                  ((size_t)max_nf * nrhs + (size_t)kST * 4) * sizeof(double), s, d, z, ldz, nrhs, T);
}
void launch_ap_et_bwd(const ApEt* d, int32_t count, const double* z, int64_t ldz, int32_t nrhs,
                      double* P, bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_et_bwd, dim3(count), dim3(kST), (size_t)kEtTileB * nrhs * sizeof(double),
                  s, d, z, ldz, nrhs, P);
}
void launch_ap_mv_rows(const ApMvTask* t, int32_t count, const ApMv* d, double* z, int64_t ldz,
                       int32_t nrhs, const double* S, double* O, bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_mv_rows, dim3(count), dim3(kApWyThreads), 0, s, t, d, z, ldz, nrhs, S, O);
}
void launch_ap_mv_cols(const ApMvTask* t, int32_t count, const ApMv* d, double* z, int64_t ldz,
                       int32_t nrhs, const double* S, double* O, bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_mv_cols, dim3(count), dim3(kApWyThreads), 0, s, t, d, z, ldz, nrhs, S, O);
}
void launch_ap_wy_dots(const ApWyTask* t, int32_t count, const ApSp* d, const double* z,
                       int64_t ldz, int32_t nrhs, const double* P, double* U, int64_t usz, int fwd,
                       bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_wy_dots, dim3(count), dim3(kApWyThreads), 0, s, t, d, z, ldz, nrhs, P, U,
                  usz, fwd);
}
void launch_ap_wy_update(const ApWyTask* t, int32_t count, const ApSp* d, double* z, int64_t ldz,
                         int32_t nrhs, const double* P, const double* U, int64_t usz, int fwd,
                         bool f32, hipStream_t s) {
  if (count <= 0) return;
  SPAND_AP_LAUNCH(f32, k_ap_wy_update, dim3(count), dim3(kApWyThreads), 0, s, t, d, z, ldz, nrhs, P,
                  U, usz, fwd);
}
void launch_ap_scale_bwd(const ApScale* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                         int32_t max_n, bool f32, hipStream_t s) {
  if (count <= 0) return;
  const size_t lds = 2 * (size_t)max_n * nrhs * sizeof(double);
  if (count >= kApNarrowFrom) {
    if (f32) hipLaunchKernelGGL((k_ap_scale_bwd<float, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
    else hipLaunchKernelGGL((k_ap_scale_bwd<double, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
  } else {
    if (f32) hipLaunchKernelGGL((k_ap_scale_bwd<float, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
    else hipLaunchKernelGGL((k_ap_scale_bwd<double, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
  }
}
void launch_ap_int_bwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       int32_t max_n, bool f32, hipStream_t s) {
  if (count <= 0) return;
  const size_t lds = ((size_t)(2 + kNW) * max_n * nrhs + (size_t)kChunk * nrhs) * sizeof(double);
  if (count >= kApNarrowFrom) {
    if (f32) hipLaunchKernelGGL((k_ap_int_bwd<float, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
    else hipLaunchKernelGGL((k_ap_int_bwd<double, kApNarrow>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
  } else {
    if (f32) hipLaunchKernelGGL((k_ap_int_bwd<float, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
    else hipLaunchKernelGGL((k_ap_int_bwd<double, kApWide>), dim3(count), dim3(kT), lds, s, d, z, ldz, nrhs);
  }
}

void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                 int32_t nrhs, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(grid_for(n, 256)), dim3(256), 0, s, rowptr, colind, vals, n, nrhs,
                     x, y);
}
int32_t dot_blocks(int32_t nseg) { return std::max(1, kDotBlocks / std::max(nseg, 1)); }

void launch_dot(const double* x, const double* y, int64_t n, int32_t nrhs, const int64_t* seg_off,
                int32_t nseg, double* partial, double* out, hipStream_t s) {
  const int bps = dot_blocks(nseg);
  hipLaunchKernelGGL(k_dot_partial, dim3(bps, nseg, nrhs), dim3(kT), 0, s, x, y, n, seg_off, partial);
  const int count = nseg * nrhs;
  hipLaunchKernelGGL(k_dot_final, dim3(count), dim3(kWave), 0, s, partial, bps, count, out);
}
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rho,
                   const double* pq, const int32_t* active, const int32_t* seg_id, int64_t n,
                   int32_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_xr, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, x, r, p, q, rho, pq,
                     active, seg_id, n, nrhs);
}
void launch_pcg_p(double* p, const double* z, double* rho, const double* rho_new,
                  const int32_t* active, const int32_t* seg_id, int64_t n, int32_t nrhs,
                  int32_t nseg, int32_t first, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_p, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, p, z, rho, rho_new,
                     active, seg_id, n, nrhs, first);
  const int count = nseg * nrhs;
  hipLaunchKernelGGL(k_copy_rho, dim3((count + 63) / 64), dim3(64), 0, s, rho, rho_new, active, count);
}
void launch_residual(const double* b, double* y, int64_t n, int32_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, b, y, n * nrhs);
}
void launch_copy_vec(const double* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_vec, dim3(grid_for(count, 256)), dim3(256), 0, s, src, dst, count);
}
void launch_prescale(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                     double* d, double* out, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, bad, INT32_MAX);
  hipLaunchKernelGGL(k_prescale_diag, dim3(grid_for(n, 256)), dim3(256), 0, s, rowptr, colind, vals,
                     n, d, bad);
  hipLaunchKernelGGL(k_prescale_vals, dim3(grid_for(n, 256)), dim3(256), 0, s, rowptr, colind, vals,
                     n, d, out);
}
void launch_scale_vec(const double* x, const double* d, double* y, int64_t n, int32_t nrhs,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_scale_vec, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, x, d, y, n,
                     n * nrhs);
}

}  // namespace spand
