// HIP kernels of the preconditioner apply and of PCG (FP64).
#include <hip/hip_runtime.h>

#include "apply.h"

namespace spand {

namespace {

constexpr int kWave = 64;
constexpr int kT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
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
// forward interior: z_s <- L^{-1} z_s ; t = G^T z_s
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_ap_int_fwd(const ApInt* descs, double* z, int64_t ldz,
                                                   int nrhs, double* T) {
  extern __shared__ double sm[];
  const ApInt d = descs[blockIdx.x];
  const int n = d.n, k = d.k;
  double* xs = sm;             // n x nrhs
  double* ys = sm + n * nrhs;  // n x nrhs
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    xs[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = 0.0;
    for (int m = 0; m <= i; ++m) acc = fma(d.Linv[i + (int64_t)m * n], xs[m + r * n], acc);
    ys[idx] = acc;
    z[d.pos[i] + r * ldz] = acc;
  }
  __syncthreads();
  if (k == 0) return;
  double* t = T + d.toff * nrhs;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int j = wid; j < k; j += kT / kWave) {
    const double* g = d.G + (int64_t)j * n;
    for (int r = 0; r < nrhs; ++r) {
      double acc = 0.0;
      for (int i = lane; i < n; i += kWave) acc = fma(g[i], ys[i + r * n], acc);
      acc = wave_sum(acc);
      if (lane == 0) t[j + (int64_t)r * k] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// gather: z_w -= sum of slices; optional scaling z_w <- Zinv z_w
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_ap_gather(const ApGat* descs, const ApSrc* src, double* z,
                                                  int64_t ldz, int nrhs, const double* T) {
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
    xs[idx] = acc;
    if (!d.Zinv) z[d.pos[i] + r * ldz] = acc;
  }
  if (!d.Zinv) return;
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = 0.0;
    for (int m = 0; m <= i; ++m) acc = fma(d.Zinv[i + (int64_t)m * n], xs[m + r * n], acc);
    z[d.pos[i] + r * ldz] = acc;
  }
}

// ---------------------------------------------------------------------------
// forward sparsification: z_p <- Q^T z_p ; t = E^T z_f
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_ap_sp_fwd(const ApSp* descs, double* z, int64_t ldz,
                                                  int nrhs, double* T) {
  extern __shared__ double sm[];
  __shared__ double red[kT / kWave];
  const ApSp d = descs[blockIdx.x];
  const int a = d.a;
  double* xs = sm;  // a x nrhs
  for (int idx = threadIdx.x; idx < a * nrhs; idx += kT) {
    const int i = idx % a, r = idx / a;
    xs[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  for (int j = 0; j < d.nref; ++j) {
    const double* v = d.V + (int64_t)j * a;
    const double tau = d.tau[j];
    for (int r = 0; r < nrhs; ++r) {
      double acc = 0.0;
      for (int i = j + threadIdx.x; i < a; i += kT) acc = fma(v[i], xs[i + r * a], acc);
      const double w = block_sum(acc, red) * tau;
      for (int i = j + threadIdx.x; i < a; i += kT) xs[i + r * a] = fma(-w, v[i], xs[i + r * a]);
      __syncthreads();
    }
  }
  for (int idx = threadIdx.x; idx < a * nrhs; idx += kT) {
    const int i = idx % a, r = idx / a;
    z[d.pos[i] + r * ldz] = xs[idx];
  }
  if (!d.E || d.f1 <= d.f0 || d.k == 0) return;
  double* t = T + d.toff * nrhs;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nf = d.f1 - d.f0;
  for (int j = wid; j < d.k; j += kT / kWave) {
    const double* e = d.E + (int64_t)j * a;  // rows f0.. of column j
    for (int r = 0; r < nrhs; ++r) {
      double acc = 0.0;
      for (int i = lane; i < nf; i += kWave) acc = fma(e[i], xs[d.f0 + i + r * a], acc);
      acc = wave_sum(acc);
      if (lane == 0) t[j + (int64_t)r * d.k] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// backward sparsification: y_f -= E y_W ; y_p <- Q y_p
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_ap_sp_bwd(const ApSp* descs, double* z, int64_t ldz,
                                                  int nrhs) {
  extern __shared__ double sm[];
  __shared__ double red[kT / kWave];
  const ApSp d = descs[blockIdx.x];
  const int a = d.a;
  double* xs = sm;
  for (int idx = threadIdx.x; idx < a * nrhs; idx += kT) {
    const int i = idx % a, r = idx / a;
    xs[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  if (d.E && d.f1 > d.f0 && d.k > 0) {
    const int nf = d.f1 - d.f0;
    for (int idx = threadIdx.x; idx < nf * nrhs; idx += kT) {
      const int i = idx % nf, r = idx / nf;
      double acc = 0.0;
      for (int j = 0; j < d.k; ++j)
        acc = fma(d.E[i + (int64_t)j * a], z[d.nbr_pos[j] + r * ldz], acc);
      xs[d.f0 + i + r * a] -= acc;
    }
    __syncthreads();
  }
  for (int j = d.nref - 1; j >= 0; --j) {
    const double* v = d.V + (int64_t)j * a;
    const double tau = d.tau[j];
    for (int r = 0; r < nrhs; ++r) {
      double acc = 0.0;
      for (int i = j + threadIdx.x; i < a; i += kT) acc = fma(v[i], xs[i + r * a], acc);
      const double w = block_sum(acc, red) * tau;
      for (int i = j + threadIdx.x; i < a; i += kT) xs[i + r * a] = fma(-w, v[i], xs[i + r * a]);
      __syncthreads();
    }
  }
  for (int idx = threadIdx.x; idx < a * nrhs; idx += kT) {
    const int i = idx % a, r = idx / a;
    z[d.pos[i] + r * ldz] = xs[idx];
  }
}

__global__ __launch_bounds__(kT) void k_ap_scale_bwd(const ApScale* descs, double* z, int64_t ldz,
                                                     int nrhs) {
  extern __shared__ double sm[];
  const ApScale d = descs[blockIdx.x];
  const int n = d.n;
  double* xs = sm;
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    xs[idx] = z[d.pos[i] + r * ldz];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = 0.0;
    for (int m = i; m < n; ++m) acc = fma(d.Zinv[m + (int64_t)i * n], xs[m + r * n], acc);
    z[d.pos[i] + r * ldz] = acc;
  }
}

// backward interior: y_s <- L^{-T} (y_s - G y_W)
__global__ __launch_bounds__(kT) void k_ap_int_bwd(const ApInt* descs, double* z, int64_t ldz,
                                                   int nrhs) {
  extern __shared__ double sm[];
  const ApInt d = descs[blockIdx.x];
  const int n = d.n, k = d.k;
  double* us = sm;
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = z[d.pos[i] + r * ldz];
    for (int j = 0; j < k; ++j) acc = fma(-d.G[i + (int64_t)j * n], z[d.nbr_pos[j] + r * ldz], acc);
    us[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += kT) {
    const int i = idx % n, r = idx / n;
    double acc = 0.0;
    for (int m = i; m < n; ++m) acc = fma(d.Linv[m + (int64_t)i * n], us[m + r * n], acc);
    z[d.pos[i] + r * ldz] = acc;
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

__global__ __launch_bounds__(kT) void k_dot_partial(const double* x, const double* y, int64_t n,
                                                    double* partial) {
  __shared__ double red[kT / kWave];
  const int r = blockIdx.y;
  const double* xr = x + r * n;
  const double* yr = y + r * n;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b = blockIdx.x * chunk, e = min(n, b + chunk);
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += kT) acc = fma(xr[i], yr[i], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x + (int64_t)r * gridDim.x] = acc;
}

__global__ void k_dot_final(const double* partial, int nparts, double* out) {
  if (threadIdx.x != 0) return;
  const int r = blockIdx.x;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += partial[i + (int64_t)r * nparts];
  out[r] = s;
}

__global__ void k_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rho,
                         const double* pq, const int32_t* active, int64_t n, int nrhs) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * nrhs;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n);
    if (!active[c]) continue;
    const double alpha = rho[c] / pq[c];
    x[idx] = fma(alpha, p[idx], x[idx]);
    r[idx] = fma(-alpha, q[idx], r[idx]);
  }
}

__global__ void k_pcg_p(double* p, const double* z, const double* rho, const double* rho_new,
                        const int32_t* active, int64_t n, int nrhs, int first) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * nrhs;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n);
    if (!active[c]) continue;
    p[idx] = first ? z[idx] : fma(rho_new[c] / rho[c], p[idx], z[idx]);
  }
}

__global__ void k_copy_rho(double* rho, const double* rho_new, const int32_t* active, int nrhs) {
  const int c = threadIdx.x;
  if (c < nrhs && active[c]) rho[c] = rho_new[c];
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

inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 16384) g = 16384;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

void launch_ap_int_fwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       double* T, int32_t max_n, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_int_fwd, dim3(count), dim3(kT), 2 * (size_t)max_n * nrhs * sizeof(double),
                     s, d, z, ldz, nrhs, T);
}
void launch_ap_gather(const ApGat* d, const ApSrc* src, int32_t count, double* z, int64_t ldz,
                      int32_t nrhs, const double* T, int32_t max_n, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_gather, dim3(count), dim3(kT), (size_t)max_n * nrhs * sizeof(double), s,
                     d, src, z, ldz, nrhs, T);
}
void launch_ap_sp_fwd(const ApSp* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                      double* T, int32_t max_a, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_sp_fwd, dim3(count), dim3(kT), (size_t)max_a * nrhs * sizeof(double), s,
                     d, z, ldz, nrhs, T);
}
void launch_ap_sp_bwd(const ApSp* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                      int32_t max_a, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_sp_bwd, dim3(count), dim3(kT), (size_t)max_a * nrhs * sizeof(double), s,
                     d, z, ldz, nrhs);
}
void launch_ap_scale_bwd(const ApScale* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                         int32_t max_n, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_scale_bwd, dim3(count), dim3(kT), (size_t)max_n * nrhs * sizeof(double),
                     s, d, z, ldz, nrhs);
}
void launch_ap_int_bwd(const ApInt* d, int32_t count, double* z, int64_t ldz, int32_t nrhs,
                       int32_t max_n, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ap_int_bwd, dim3(count), dim3(kT), (size_t)max_n * nrhs * sizeof(double), s,
                     d, z, ldz, nrhs);
}

void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* vals, int64_t n,
                 int32_t nrhs, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(grid_for(n, 256)), dim3(256), 0, s, rowptr, colind, vals, n, nrhs,
                     x, y);
}
void launch_dot(const double* x, const double* y, int64_t n, int32_t nrhs, double* partial,
                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks, nrhs), dim3(kT), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(64), 0, s, partial, kDotBlocks, out);
}
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rho,
                   const double* pq, const int32_t* active, int64_t n, int32_t nrhs,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_xr, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, x, r, p, q, rho, pq,
                     active, n, nrhs);
}
void launch_pcg_p(double* p, const double* z, double* rho, const double* rho_new,
                  const int32_t* active, int64_t n, int32_t nrhs, int32_t first, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_p, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, p, z, rho, rho_new,
                     active, n, nrhs, first);
  hipLaunchKernelGGL(k_copy_rho, dim3(1), dim3(64), 0, s, rho, rho_new, active, nrhs);
}
void launch_residual(const double* b, double* y, int64_t n, int32_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, b, y, n * nrhs);
}
void launch_copy_vec(const double* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_vec, dim3(grid_for(count, 256)), dim3(256), 0, s, src, dst, count);
}

}  // namespace spand
