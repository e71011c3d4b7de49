// Cooperative early-stopping column-pivoted Householder QR (Alg. 1) with the
// coupling W (a x k) of one interface held in registers.
//
// A group of G workgroups shares the columns of W, at most 64 per workgroup:
// each 8-lane group of a wave owns one column, lane r of the group holds rows
// r, r + 8, r + 16, ... (R rows, a <= 8R).  A pivot step is then
//   1. local maximum of the trailing norms and the ordered list of local tie
//      candidates; the group of the first candidate publishes its column;
//   2. one group barrier (inside one XCD's L2, see kernels_qr_coop.hip);
//   3. one round of loads: every workgroup fetches all G lists and all G
//      published columns, picks the global pivot (lowest index among the
//      columns within the tie band of the global maximum) and finds its column
//      among the published ones (a second round covers the rare cases where
//      the lists overflow or the pivot is not its owner's first candidate);
//   4. the Householder reflector is applied to every column in registers, with
//      an 8-lane reduction for the dot product and another for the exact new
//      trailing norm.
// The pivot sequence, stopping rule and outputs are those of k_cpqr_coop.
#include <climits>

#include "device.h"

namespace spand {

namespace {

constexpr int kWave = 64;
constexpr int kRT = 512;                 // threads per workgroup (256 VGPRs per lane)
constexpr int kRW = kRT / kWave;         // waves per workgroup
constexpr int kList = 32;                // tie candidates published per workgroup
constexpr int kXs = 2 + 2 * kList;       // exchange stride: max, count, idx[], nrm2[]
constexpr long kSpinLimit = 1L << 24;

template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int kCtrl>
__device__ __forceinline__ double dpp_move_ninf(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)0xfff00000, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move_ninf<0xb1>(v));
  v = fmax(v, dpp_move_ninf<0x4e>(v));
  v = fmax(v, dpp_move_ninf<0x124>(v));
  v = fmax(v, dpp_move_ninf<0x128>(v));
  v = fmax(v, dpp_move_ninf<0x142>(v));
  v = fmax(v, dpp_move_ninf<0x143>(v));
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// values that are the same in every lane, moved to scalar registers
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

__device__ __forceinline__ int xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xf;
}
__device__ __forceinline__ void xst(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ double xld(const double* p) {
  const unsigned long long u = __hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(u));
}

__device__ bool group_barrier(int32_t* flags, int phase, int G, int g, int32_t* err, int* sok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (G == 1) return true;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    if (lane == 0) __hip_atomic_store(flags + g, phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    long spins = 0;
    int ok = 1;
    while (true) {
      const int f = lane < G
                        ? __hip_atomic_load(flags + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : phase;
      if (__all(f >= phase)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        ok = 0;
        if (lane == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    if (lane == 0) *sok = ok;
  }
  __syncthreads();
  return *sok != 0;
}

template <int R>
__global__ __launch_bounds__(kRT) void k_cpqr_reg(const CoopDesc* descs, const CpqrNbr* nbrs,
                                                 const int32_t* blk_map, int32_t* n_cur,
                                                 int32_t* out_r, int32_t* out_r2, int32_t* out_k,
                                                 double eps, double eps_stop, int32_t* err) {
  extern __shared__ double sm[];
  __shared__ double red_max[kRW], red_M[kRW];
  __shared__ int red_over[kRW], red_C[kRW], red_C2[kRW], s_wcnt[kRW];
  __shared__ int sok, sC, sover;
  __shared__ double sM;
  const int code = blk_map[blockIdx.x];
  if (code < 0) return;   // idle slot of the XCD packing
  const CoopDesc cd = descs[code / kCoopMaxGroup];
  const CpqrDesc& d = cd.d;
  const int G = cd.G, g = code % kCoopMaxGroup;
  const int a = d.a;
  const int64_t K = d.kmax;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int grp = lane >> 3, r8 = lane & 7;
  int32_t* flags = cd.sync + kCoopFlag0;

  if (tid == 0) {
    int ok = 1, loc = 1;
    if (G > 1) {
      const int mine = 1 + ((cd.xcd >= 0 && xcc_id() == cd.xcd) ? 0 : (1 << 16));
      __hip_atomic_fetch_add(cd.sync, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      long spins = 0;
      int cnt;
      while (((cnt = __hip_atomic_load(cd.sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
              0xffff) < G) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          ok = 0;
          __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      loc = ok && (cnt >> 16) == 0;
      if (ok && !loc) __hip_atomic_fetch_or(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sok = ok && loc;
  }
  __syncthreads();
  if (!sok) return;   // timed out, or not on one XCD: nothing has been written

  int k = 0;
  for (int64_t e = d.nb0; e < d.nb1; ++e) k += n_cur[nbrs[e].w];
  const int per = (k + G - 1) / G;
  const int c0 = min(k, g * per), c1 = min(k, c0 + per), m = c1 - c0;
  const int c = wid * 8 + grp;          // my column (local index)
  const bool mine = c < m;
  const int gc = c0 + c;                // its index in W

  // LDS: published columns of the G workgroups (slot q: norm^2, rows j..a-1)
  double* Pc = sm;                      // G x (a + 1)
  int* heads = reinterpret_cast<int*>(Pc + (int64_t)G * (a + 1));   // G list heads
  double* X2 = cd.xch;
  double* PV2 = X2 + 2 * (int64_t)G * kXs;
  double* PVx = PV2 + 2 * (int64_t)G * (a + 1);
  double* XB = PVx + a + 1;

  // my column of W: block (p, w) of p's panel, and (w, p) of w's panel
  const double* src = nullptr;
  double* dst_wp = nullptr;
  int ldw = 0;
  if (mine) {
    int kk = 0;
    for (int64_t e = d.nb0; e < d.nb1; ++e) {
      const CpqrNbr nb = nbrs[e];
      const int wc = n_cur[nb.w];
      if (gc < kk + wc) {
        const int cw = gc - kk;
        src = d.panel + (nb.col + cw) * a;
        dst_wp = nb.blk_wp + cw;
        ldw = nb.ldw;
        break;
      }
      kk += wc;
    }
  }
  double y[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = r8 + 8 * t;
    y[t] = (mine && i < a) ? src[i] : 0.0;
  }
  double nrm;
  {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) s = fma(y[t], y[t], s);
    s = group8_sum(s);
    nrm = mine ? s : -1.0;
  }

  int phase = 0;
  int r = -1, j = 0;
  double R00 = 0.0;
  const int jmax = min(a, k);
  for (; j < jmax; ++j) {
    double* X = X2 + (int64_t)(j & 1) * G * kXs;
    double* PVs = PV2 + (int64_t)(j & 1) * G * (a + 1);
    // ---- 1. local maximum and ordered tie candidates ----
    {
      const double ml = wave_max(nrm);
      if (lane == 0) red_max[wid] = ml;
    }
    __syncthreads();
    // per-wave partials are reduced with one LDS read per lane and a wave reduction
    const double Mg = uni(wave_max(lane < kRW ? red_max[lane] : -HUGE_VAL));
    const double thl = Mg * (1.0 - kPivotTieRtol);
    const bool f = Mg >= 0.0 && nrm >= 0.0 && nrm >= thl;
    const unsigned long long mask = __ballot(f && r8 == 0);
    if (lane == 0) s_wcnt[wid] = __popcll(mask);
    __syncthreads();
    const int cnt_l = lane < kRW ? s_wcnt[lane] : 0;
    const int total = uni(wave_sum_int(cnt_l));
    const int before = uni(wave_sum_int(lane < wid ? cnt_l : 0));
    double* Xg = X + (int64_t)g * kXs;
    const int at = before + __popcll(mask & ((1ULL << (lane & ~7)) - 1ULL));
    if (f && r8 == 0 && at < cd.list_cap) {
      xst(Xg + 2 + at, (double)gc);
      xst(Xg + 2 + kList + at, nrm);
    }
    if (f && at == 0) {   // first candidate: publish its column
      double* Pg = PVs + (int64_t)g * (a + 1);
      if (r8 == 0) xst(Pg, nrm);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = r8 + 8 * t;
        if (i >= j && i < a) xst(Pg + 1 + (i - j), y[t]);
      }
    }
    if (tid == 0) {
      xst(Xg, Mg);
      xst(Xg + 1, (double)total);
    }
    // ---- 2. group barrier ----
    if (!group_barrier(flags, ++phase, G, g, err, &sok)) return;
    // ---- 3. one round of loads: all lists and all published columns ----
    constexpr int kSlots = (kCoopMaxGroup * kList + kRT - 1) / kRT;
    double nv[kSlots];
    int ix[kSlots], cq[kSlots];
    double Mloc = -2.0;
    int ovl = 0;
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const int idx = tid + u * kRT, q = idx / kList, e = idx % kList;
      nv[u] = -1.0;
      ix[u] = INT_MAX;
      cq[u] = 0;
      if (q < G) {
        const double* Xq = X + (int64_t)q * kXs;
        const double Mq = xld(Xq);
        cq[u] = (int)xld(Xq + 1);
        if (e < cd.list_cap) {
          ix[u] = (int)xld(Xq + 2 + e);
          nv[u] = xld(Xq + 2 + kList + e);
        }
        Mloc = fmax(Mloc, Mq);
        if (e == 0) {
          ovl |= cq[u] > cd.list_cap ? 1 : 0;
          heads[q] = (cq[u] > 0 && cd.list_cap > 0) ? ix[u] : -1;
        }
      }
    }
    const int len = a - j + 1;
    for (int idx = tid; idx < G * len; idx += kRT) {
      const int qq = idx / len, ii = idx - qq * len;
      Pc[(int64_t)qq * (a + 1) + ii] = xld(PVs + (int64_t)qq * (a + 1) + ii);
    }
    {
      const double mm = wave_max(Mloc);
      const int ov = wave_max_int(ovl);
      if (lane == 0) {
        red_M[wid] = mm;
        red_over[wid] = ov;
      }
    }
    __syncthreads();
    const double M = uni(wave_max(lane < kRW ? red_M[lane] : -HUGE_VAL));
    const int over = uni(wave_max_int(lane < kRW ? red_over[lane] : 0));
    if (M < 0.0) break;   // every column used up (uniform)
    const double thr = M * (1.0 - kPivotTieRtol);
    int C = INT_MAX;
    if (!over) {
#pragma unroll
      for (int u = 0; u < kSlots; ++u) {
        const int e = (tid + u * kRT) % kList;
        if (e < cq[u] && nv[u] >= thr) C = min(C, ix[u]);
      }
    } else {
      // exact local candidates against the global threshold
      const bool cand = nrm >= 0.0 && nrm >= thr && r8 == 0;
      const unsigned long long cm = __ballot(cand);
      int cl = cm ? c0 + wid * 8 + (__ffsll((long long)cm) - 1) / 8 : INT_MAX;
      if (lane == 0) red_C[wid] = cl;
      __syncthreads();
      if (wid == 0) {
        const int mn = wave_min_int(lane < kRW ? red_C[lane] : INT_MAX);
        if (lane == 0) xst(XB + g, (double)mn);
      }
      if (!group_barrier(flags, ++phase, G, g, err, &sok)) return;
      for (int qq = tid; qq < G; qq += kRT) C = min(C, (int)xld(XB + qq));
    }
    C = wave_min_int(C);
    if (lane == 0) red_C2[wid] = C;
    __syncthreads();
    C = uni(wave_min_int(lane < kRW ? red_C2[lane] : INT_MAX));
    const int og = min(C / max(per, 1), G - 1);   // owner workgroup
    const bool spec = !over && uni(heads[og]) == C;
    const double* PV = Pc + (int64_t)og * (a + 1);
    if (!spec) {
      // the owner publishes the pivot column; everybody loads it into slot og
      if (mine && gc == C) {
        if (r8 == 0) xst(PVx, nrm);
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = r8 + 8 * t;
          if (i >= j && i < a) xst(PVx + 1 + (i - j), y[t]);
        }
      }
      if (!group_barrier(flags, ++phase, G, g, err, &sok)) return;
      for (int ii = tid; ii < len; ii += kRT) Pc[(int64_t)og * (a + 1) + ii] = xld(PVx + ii);
      __syncthreads();
    }
    // ---- 4. reflector ----
    const double pn = uni(PV[0]), alpha = uni(PV[1]);
    const double pnrm = sqrt(pn);
    if (j == 0) R00 = pnrm;
    if (pnrm == 0.0 || pnrm < eps_stop * R00) break;
    if (r < 0 && pnrm < eps * R00) r = j;
    const double beta = alpha >= 0.0 ? -pnrm : pnrm;
    const double rden = 1.0 / (alpha - beta);
    const double tau = (beta - alpha) / beta;
    if (g == 0) {
      for (int i = tid; i < a; i += kRT)
        d.V[i + (int64_t)j * a] = i < j ? 0.0 : (i == j ? 1.0 : PV[1 + (i - j)] * rden);
      if (tid == 0) d.tau[j] = tau;
    }
    const bool piv = mine && gc == C;
    const bool act = mine && nrm >= 0.0 && !piv;
    // branch-free over the rows of this lane: v_i = 0 outside j..a-1, so
    // rows above j and padding rows are left unchanged by the update
    const double* Pv = PV + 1;
    double dot = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = r8 + 8 * t;
      const double raw = Pv[min(max(i - j, 0), a - 1)];
      const double vi = (i > j && i < a) ? raw * rden : (i == j ? 1.0 : 0.0);
      dot = fma(vi, y[t], dot);
    }
    dot = group8_sum(dot) * tau;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = r8 + 8 * t;
      const double raw = Pv[min(max(i - j, 0), a - 1)];
      const double vi = (i > j && i < a) ? raw * rden : (i == j ? 1.0 : 0.0);
      const double yn = fma(-dot, vi, y[t]);
      const double yt = i > j ? yn : 0.0;
      s = fma(yt, yt, s);
      const double ypiv = i == j ? beta : (i > j ? 0.0 : y[t]);
      y[t] = act ? yn : (piv ? ypiv : y[t]);
    }
    s = group8_sum(s);
    if (act) nrm = s;
    if (piv) nrm = -1.0;
  }
  const int nref = j;
  if (r < 0) r = nref;

  if (mine) {
    // Q^T W into the transposed workspace; coarse rows into p's panel and,
    // transposed, into the neighbour's panel
    double* pcol = const_cast<double*>(src);
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = r8 + 8 * t;
      if (i < a) d.Y[gc + (int64_t)i * K] = y[t];
      if (i < r) {
        pcol[i] = y[t];
        dst_wp[(int64_t)i * ldw] = y[t];
      }
    }
  }
  if (g != 0) return;
  for (int idx = tid; idx < r * r; idx += kRT) {
    const int i = idx % r, cc = idx / r;
    d.panel[i + (d.diag_col + cc) * a] = i == cc ? 1.0 : 0.0;
  }
  if (tid == 0) {
    out_k[d.p] = k;
    out_r[d.p] = r;
    out_r2[d.p] = nref;
    n_cur[d.p] = r;
  }
}

}  // namespace

int cpqr_reg_rows(int a) {
  return a <= 96 ? 12 : a <= 160 ? 20 : a <= 224 ? 28 : a <= kCpqrRegMaxA ? 36 : 0;
}

size_t cpqr_reg_lds(int G, int a) {
  return (size_t)G * (a + 1) * sizeof(double) + (size_t)G * sizeof(int);
}

int cpqr_reg_max_blocks(int rows, size_t lds_bytes) {
  int dev = 0, ncu = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = rows == 12   ? reinterpret_cast<const void*>(k_cpqr_reg<12>)
                   : rows == 20 ? reinterpret_cast<const void*>(k_cpqr_reg<20>)
                   : rows == 28 ? reinterpret_cast<const void*>(k_cpqr_reg<28>)
                                : reinterpret_cast<const void*>(k_cpqr_reg<36>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kRT, lds_bytes) != hipSuccess) return 0;
  return nb * ncu;
}

hipError_t launch_cpqr_reg(int rows, const CoopDesc* d, const CpqrNbr* nb, const int32_t* blk_map,
                           int32_t nblocks, int32_t* sync, int32_t nsync, int32_t* n_cur,
                           int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps,
                           double eps_stop, int32_t* err, size_t lds_bytes, hipStream_t s) {
  launch_fill_int(sync, nsync, s);
  void* args[] = {(void*)&d, (void*)&nb, (void*)&blk_map, (void*)&n_cur, (void*)&out_r,
                  (void*)&out_r2, (void*)&out_k, (void*)&eps, (void*)&eps_stop, (void*)&err};
  const void* fn = rows == 12   ? reinterpret_cast<const void*>(k_cpqr_reg<12>)
                   : rows == 20 ? reinterpret_cast<const void*>(k_cpqr_reg<20>)
                   : rows == 28 ? reinterpret_cast<const void*>(k_cpqr_reg<28>)
                                : reinterpret_cast<const void*>(k_cpqr_reg<36>);
  return hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(kRT), args, lds_bytes, s);
}

}  // namespace spand
