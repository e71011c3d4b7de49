// Cooperative early-stopping column-pivoted Householder QR (Alg. 1): the
// coupling W (a x k) of one interface is split by columns over a group of G
// workgroups, each holding its column slice in LDS for the whole
// factorization.  A pivot step is a serial chain run by wave 0 of every
// workgroup, then a parallel update by all waves:
//
//  A. wave 0 finds its largest trailing norm and the ordered list of its
//     columns within the tie band of that maximum, publishes both and the
//     column of its first candidate, and meets the other workgroups at a group
//     barrier whose flag words also carry each maximum (as float) and first
//     candidate: when one group's maximum exceeds all others by more than
//     float rounding, far more than the band, the pivot is that group's first
//     candidate and no further round is needed.  Otherwise, since the global
//     band lies inside every local band, the union
//     of the lists holds every global candidate, and each workgroup picks the
//     same pivot (lowest index among the columns within the band of the global
//     maximum).  If a list overflows, an extra round exchanges exact local
//     candidates; if the pivot is not its owner's first candidate, the owner
//     publishes it in an extra round.  Wave 0 then builds the Householder
//     vector in LDS.
//  C. every wave updates its columns and recomputes their trailing norms
//     exactly (8 lanes per column, one DPP reduction for the dot product and
//     one for the norm).
//
// One workgroup alone (G = 1) skips the exchange and reads the pivot from LDS.
// A workgroup may belong to several groups in turn: the groups of one colour
// that do not fit the co-resident workgroups together are packed in rounds,
// and one launch runs all rounds, each workgroup starting its group of the
// next round as soon as it is done with the previous one (its LDS slice,
// norms and barrier state are set up afresh for every group).
// Synchronization.  The launcher plans all workgroups of a group on one XCD
// (planned block b on XCD b mod 8), and a workgroup takes the next planned
// block of the XCD it actually runs on (the grid fills every compute unit, so
// every XCD holds the same number of workgroups in whatever order the hardware
// places them).  The group then exchanges data through that XCD's L2: plain stores (the CU's L1 is write-through) and
// agent-scope loads (which miss the L1), with barrier flags polled the same
// way.  At entry every workgroup checks its XCD against the planned one with
// one round of device-coherent atomics; a group that is not on one XCD leaves
// before writing anything and raises bit 2 of the error flag, and the host
// then redoes the factorization with the single-workgroup QR.  The launch is
// cooperative (all workgroups resident) and every spin is bounded: a timeout
// raises bit 1 of the error flag and all workgroups leave.
#include <climits>

#include "device.h"

namespace spand {

namespace {

constexpr int kWave = 64;
constexpr int kCT = 1024;               // threads per workgroup
constexpr int kCW = kCT / kWave;        // waves per workgroup
constexpr int kList = kCoopList;        // tie candidates published per workgroup
constexpr int kXs = 2 + 2 * kList;      // exchange stride: max, count, idx[], nrm2[]
constexpr long kSpinLimit = 1L << 24;   // ~ seconds of s_sleep before giving up
constexpr int kRpl = 4;                 // rows per lane kept in registers by the update (8 lanes
constexpr int kRpl16 = 4;               // per column); with 16 and 32 lanes per column
constexpr int kRpl32 = 4;
constexpr int kUnrollLds = 4;           // loads in flight per lane in the update's other rows
constexpr int kUnrollPanel = 8;         // (LDS slice; panel columns in global memory)
constexpr int kPv = 4;                  // pivot-column entries per lane loaded at once
constexpr int kScan = 2;                // column norms per lane held by the pivot scan

template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1>(v);
  v += dpp_move<0x4e>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x128>(v);
  v += dpp_move<0x142>(v);
  v += dpp_move<0x143>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over each group of 8 lanes, returned to all 8: two quad permutations and
// a half-row mirror.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  return v;
}

template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xb1>(v);
  v += dpp_move<0x4e>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x128>(v);
  v += dpp_move<0x142>(v);
  v += dpp_move<0x143>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// threadIdx.x through an opaque move: in the membership loop of the
// cooperative QR the compiler would otherwise compute every value derived
// from it once, before the loop, and keep it live across the whole body
// (register spills in the pivot steps); this way they are recomputed where
// they are used
__device__ __forceinline__ int tid_x() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

// Sum over each group of L lanes (8, 16, 32 or 64), returned to all of them.
template <int L, class R>
__device__ __forceinline__ R groupL_sum(R v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  if (L == 8) {
    v += dpp_move<0x141>(v);  // row_half_mirror
  } else {
    v += dpp_move<0x124>(v);  // row_ror:4
    v += dpp_move<0x128>(v);  // row_ror:8
    if (L >= 32) v += __shfl_xor(v, 16, kWave);
    if (L == 64) v += __shfl_xor(v, 32, kWave);
  }
  return v;
}

// Reflector update and exact trailing norms of m columns of one workgroup
// (in the LDS slice Ys, ld a, or, kPanel, at the addresses gcol in the row
// panel): L lanes per column (64 / L columns per wave, the
// waves over the column batches), kRpl rows per lane held in registers between
// the dot product and the update, one group reduction for each.  Column Cl
// (the pivot, when owned) and used-up columns (nrm2 < 0) are skipped.
template <int L, int kRpl, bool kPanel, class R>
__device__ __forceinline__ void update_columns(R* Ys, R* const* gcol, R* nrm2, const R* v, int a,
                                               int m, int j, R tau, int skip) {
  constexpr int CPW = kWave / L;   // columns per wave
  constexpr int kU = kPanel ? kUnrollPanel : kUnrollLds;
  const int tx = tid_x(), lane = tx & (kWave - 1), wid = tx / kWave;
  const int grp = lane / L, rl = lane % L;
  for (int cb = wid * CPW; cb < m; cb += kCW * CPW) {
    const int c = cb + grp;
    const bool act = c < m && c != skip && nrm2[c] >= R(0);
    // LDS slice, or (kPanel) the column's place in the panel
    R* col = kPanel ? (act ? gcol[c] : gcol[0]) : Ys + (int64_t)(act ? c : 0) * a;
    R yv[kRpl];
    R dot = 0;
#pragma unroll
    for (int t = 0; t < kRpl; ++t) {
      const int i = j + rl + L * t;
      const bool in = act && i < a;
      yv[t] = in ? col[i] : R(0);
      dot = fma(in ? v[i] : R(0), yv[t], dot);
    }
    // rows beyond the register block: kU rows' loads in flight per lane
    // (more for panel columns, which live in global memory), accumulated in
    // the same order
    const int i4 = j + rl + L * kRpl;
    if (act) {
      int i = i4;
      for (; i + (kU - 1) * L < a; i += kU * L) {
        R vr[kU], wr[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          vr[u] = v[i + u * L];
          wr[u] = col[i + u * L];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) dot = fma(vr[u], wr[u], dot);
      }
      for (; i < a; i += L) dot = fma(v[i], col[i], dot);
    }
    dot = groupL_sum<L>(dot) * tau;
    R s = 0;
#pragma unroll
    for (int t = 0; t < kRpl; ++t) {
      const int i = j + rl + L * t;
      if (act && i < a) {
        const R y = fma(-dot, v[i], yv[t]);
        col[i] = y;
        if (i > j) s = fma(y, y, s);
      }
    }
    if (act) {
      int i = i4;
      for (; i + (kU - 1) * L < a; i += kU * L) {
        R vr[kU], wr[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          vr[u] = v[i + u * L];
          wr[u] = col[i + u * L];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const R y = fma(-dot, vr[u], wr[u]);
          col[i + u * L] = y;
          s = fma(y, y, s);
        }
      }
      for (; i < a; i += L) {
        const R y = fma(-dot, v[i], col[i]);
        col[i] = y;
        s = fma(y, y, s);
      }
    }
    s = groupL_sum<L>(s);
    if (act && rl == 0) nrm2[c] = s;
  }
}

// DPP move whose invalid source lanes read -inf (for maxima)
template <int kCtrl>
__device__ __forceinline__ double dpp_move_ninf(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)0xfff00000, __double2hiint(x), kCtrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
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

// DPP move of a 32-bit value whose invalid source lanes read `fill`
template <int kCtrl>
__device__ __forceinline__ int dpp_move_i32(int x, int fill) {
  return __builtin_amdgcn_update_dpp(fill, x, kCtrl, 0xf, 0xf, false);
}

// minimum over the wave, returned to every lane (same DPP pattern as wave_max)
__device__ __forceinline__ int wave_min_int(int v) {
  v = min(v, dpp_move_i32<0xb1>(v, INT_MAX));
  v = min(v, dpp_move_i32<0x4e>(v, INT_MAX));
  v = min(v, dpp_move_i32<0x124>(v, INT_MAX));
  v = min(v, dpp_move_i32<0x128>(v, INT_MAX));
  v = min(v, dpp_move_i32<0x142>(v, INT_MAX));
  v = min(v, dpp_move_i32<0x143>(v, INT_MAX));
  return __builtin_amdgcn_readlane(v, 63);
}

// XCD this wave runs on (hardware register XCC_ID, bits 3:0)
__device__ __forceinline__ int xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xf;
}

// exchange stores: plain stores, which land in the XCD's L2 (the L1 is write-through)
__device__ __forceinline__ void xst(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_WORKGROUP);
}
// exchange loads bypass the CU's L1
__device__ __forceinline__ double xld(const double* p) {
  const unsigned long long u = __hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(u));
}

// Group barrier on per-member 64-bit flags, run by one wave (the only one that
// writes exchange data): it waits for its own exchange stores, then writes its
// flag word (phase in bits 63..48, a 48-bit payload below) and polls the G
// words of the same phase parity (one load per lane) until all carry the
// phase.  Flags are double buffered by phase parity: a member can be at most
// one barrier ahead of a slow reader, so the word a reader sees for phase p is
// the one written for p.  Lane q returns member q's word.  Returns false after
// a timeout (bit 1 of the error flag set).
//
// Ordering.  Every member of a group runs on one XCD (checked at kernel
// entry), so the XCD's L2 is the point where all of them see the same memory:
// a store leaves the CU through its write-through L1 and completes in that L2,
// and the exchange loads (agent scope) skip the L1 and read that L2.  The
// writer waits for its data stores to complete (s_waitcnt) before it issues
// the flag store, so a reader that sees the flag sees the data; a reader's
// data loads are issued after its poll has returned the flag.  The two
// workgroup-scope fences only keep the compiler from moving memory accesses
// across the flag store and the poll (they add no cache maintenance); an
// agent-scope release or acquire would instead write back or invalidate the
// whole L2 on every barrier, which the XCD-local placement makes unnecessary.
__device__ bool wave_barrier(unsigned long long* flags, int phase, unsigned long long payload, int G,
                             int g, int32_t* err, unsigned long long* word) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);   // this wave's exchange stores have completed
  const int lane = tid_x() & (kWave - 1);
  unsigned long long* f = flags + (phase & 1) * kCoopMaxGroup;
  const unsigned long long mine =
      ((unsigned long long)phase << 48) | (payload & 0xFFFFFFFFFFFFull);
  if (lane == 0) __hip_atomic_store(f + g, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  long spins = 0;
  while (true) {
    const unsigned long long w =
        lane < G ? __hip_atomic_load(f + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : mine;
    if (__all((int)(w >> 48) == phase)) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      *word = w;
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      if (lane == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// maximum over the wave, returned to every lane (invalid DPP sources read -inf)
__device__ __forceinline__ float wave_max_f(float v) {
  constexpr int kNinf = (int)0xff800000;
  v = fmaxf(v, __int_as_float(dpp_move_i32<0xb1>(__float_as_int(v), kNinf)));
  v = fmaxf(v, __int_as_float(dpp_move_i32<0x4e>(__float_as_int(v), kNinf)));
  v = fmaxf(v, __int_as_float(dpp_move_i32<0x124>(__float_as_int(v), kNinf)));
  v = fmaxf(v, __int_as_float(dpp_move_i32<0x128>(__float_as_int(v), kNinf)));
  v = fmaxf(v, __int_as_float(dpp_move_i32<0x142>(__float_as_int(v), kNinf)));
  v = fmaxf(v, __int_as_float(dpp_move_i32<0x143>(__float_as_int(v), kNinf)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <class R>
__device__ __forceinline__ R wave_max_r(R v) {
  if constexpr (sizeof(R) == 8) return wave_max(v);
  else return wave_max_f(v);
}

// 64-bit value of a lane given by a wave-uniform index
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// kPanel: some columns of a workgroup may live in the row panel (an interface
// wider than its group's LDS); the LDS-only instance keeps its registers for
// the common case.
template <class R, bool kPanel>
__global__ __launch_bounds__(kCT) void k_cpqr_coop(const CoopDescT<R>* descs, const CpqrNbrT<R>* nbrs,
                                                  const int32_t* blk_map, const int32_t* blk_ptr,
                                                  int32_t nplan, int32_t* xcd_slot,
                                                  int32_t* n_cur, int32_t* out_r, int32_t* out_r2,
                                                  int32_t* out_k, double eps, double eps_stop,
                                                  int32_t* err) {
  extern __shared__ __align__(16) char smraw[];
  R* sm = reinterpret_cast<R*>(smraw);
  __shared__ int sok, sC, s_go, s_r, s_vb;
  __shared__ double s_beta, s_tau;
  // The planned block b = xcd + 8 * slot: this workgroup takes the next slot
  // of the XCD it runs on.  The grid fills every compute unit, so each XCD
  // holds the same number of workgroups whatever order the hardware places
  // them in, and every planned block index below nplan is taken once.
  if (threadIdx.x == 0) {
    const int x = xcc_id();
    s_vb = x < kCoopXcds
               ? x + kCoopXcds * __hip_atomic_fetch_add(xcd_slot + x, 1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
               : INT_MAX;
  }
  __syncthreads();
  const int vb = s_vb;
  // the group memberships of this workgroup, run in order: blk_map[vb]
  // alone, or (blk_ptr) blk_map[blk_ptr[vb] .. blk_ptr[vb + 1]); none beyond
  // the planned blocks
  const int t0 = vb >= nplan ? 0 : blk_ptr ? blk_ptr[vb] : vb;
  const int t1 = vb >= nplan ? 0 : blk_ptr ? blk_ptr[vb + 1] : vb + 1;
  for (int t = t0; t < t1; ++t) {
    const int code = blk_map[t];
    if (code < 0) continue;   // idle slot of the XCD packing
    __syncthreads();          // the previous membership's epilogue is done with the LDS
    const CoopDescT<R> cd = descs[code / kCoopMaxGroup];
    const CpqrDescT<R>& d = cd.d;
    const int G = cd.G, g = code % kCoopMaxGroup;
    const int a = d.a;
    const int64_t K = d.kmax;
    const int tid = tid_x(), lane = tid & (kWave - 1), wid = tid / kWave;
    unsigned long long* flags = reinterpret_cast<unsigned long long*>(cd.sync + kCoopFlag64);
    unsigned long long bw = 0;   // flag words of the last barrier (lane q: member q)

    // placement check: one round of device-coherent atomics on sync[0] (low
    // half counts arrivals, high half counts members off the planned XCD)
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
      sok = !ok ? -1 : loc;
    }
    __syncthreads();
    // not on one XCD: the group leaves before writing anything (its members go
    // on with their next groups, which check their own placement); timed out:
    // the workgroup leaves
    if (sok < 0) return;
    if (sok == 0) continue;

    int k = 0;
    for (int64_t e = d.nb0; e < d.nb1; ++e) k += n_cur[nbrs[e].w];
    const int per = (k + G - 1) / G;
    const int c0 = min(k, g * per), c1 = min(k, c0 + per), m = c1 - c0;
    // the first mL of my columns in LDS, the rest (when the interface is wider
    // than the group's LDS) in place in the row panel
    const int mL = kPanel ? min(m, cd.ncap_lds) : m;
    R* Ys = sm;                                       // a x ncap_lds (ld a)
    R* nrm2 = sm + (int64_t)a * cd.ncap_lds;          // ncap
    R* v = nrm2 + cd.ncap;                            // a
    // ncap - ncap_lds panel column addresses, 8-byte aligned after v
    R** gcol = reinterpret_cast<R**>(smraw + coop_lds_ptr_offset<R>(a, cd.ncap, cd.ncap_lds));
    auto colp = [&](int c) -> R* {
      if constexpr (kPanel) return c < mL ? Ys + (int64_t)c * a : gcol[c - mL];
      return Ys + (int64_t)c * a;
    };
    // exchange: lists and first-candidate columns are double buffered by step
    // parity (a workgroup may publish step j+1 while others still read step j)
    double* X2 = cd.xch;                              // 2 x G x kXs
    double* PV2 = X2 + 2 * (int64_t)G * kXs;          // 2 x G x (a + 1)
    double* PVx = PV2 + 2 * (int64_t)G * (a + 1);     // a + 1: pivot of the slow path
    double* XB = PVx + a + 1;                         // G

    // my columns [c0, c1) of W
    {
      int kk = 0;
      for (int64_t e = d.nb0; e < d.nb1; ++e) {
        const CpqrNbrT<R> nb = nbrs[e];
        const int wc = n_cur[nb.w];
        const int lo = max(kk, c0), hi = min(kk + wc, c1);
        const int hiL = min(hi, c0 + mL);
        if (hiL > lo) {
          const R* src = d.panel + (nb.col + (lo - kk)) * a;
          R* dst = Ys + (int64_t)(lo - c0) * a;
          for (int idx = tid; idx < (hiL - lo) * a; idx += kCT) dst[idx] = src[idx];
        }
        if (kPanel)
          for (int c = max(lo, c0 + mL) + tid; c < hi; c += kCT)
            gcol[c - c0 - mL] = d.panel + (nb.col + (c - kk)) * a;
        kk += wc;
      }
    }
    __syncthreads();
    for (int c = wid; c < m; c += kCW) {
      const R* col = colp(c);
      R s = 0;
      for (int i = lane; i < a; i += kWave) s = fma(col[i], col[i], s);
      s = wave_sum(s);
      if (lane == 0) nrm2[c] = s;
    }
    if (tid == 0) s_r = -1;
    __syncthreads();

    // Per pivot step the serial chain runs in wave 0 alone (local maximum and
    // ordered candidate list from nrm2, publishing, the group barrier, the
    // global decision, the pivot column and the reflector into LDS); every wave
    // then updates its columns.  Two workgroup barriers per step.
    int phase = 0;
    int r = -1, j = 0;
    double R00 = 0.0;
    const int jmax = min(a, k);
    for (; j < jmax; ++j) {
      if (wid == 0) {
        int go = 1;
        // ---- local maximum and the ordered list of local tie candidates ----
        // (the norms of the first kScan * 64 columns read once, into registers)
        R nv[kScan];
        R ml = -1;
  #pragma unroll
        for (int t = 0; t < kScan; ++t) {
          const int c = lane + t * kWave;
          nv[t] = c < m ? nrm2[c] : R(-1);
          ml = fmax(ml, nv[t]);
        }
        for (int c = lane + kScan * kWave; c < m; c += kWave) ml = fmax(ml, nrm2[c]);
        const R Mg = wave_max_r(ml);
        const R thl = Mg * R(1.0 - PivotTie<R>::rtol);
        double* X = X2 + (int64_t)(j & 1) * G * kXs;
        double* PVs = PV2 + (int64_t)(j & 1) * G * (a + 1);
        double* Xg = X + (int64_t)g * kXs;
        int total = 0, first = -1;
        auto chunk = [&](const int cb, const R x) {
          const int c = cb + lane;
          const bool f = Mg >= R(0) && c < m && x >= R(0) && x >= thl;
          const unsigned long long mask = __ballot(f);
          if (f && G > 1) {
            const int at = total + __popcll(mask & ((1ULL << lane) - 1ULL));
            if (at < cd.list_cap) {
              xst(Xg + 2 + at, (double)(c0 + c));
              xst(Xg + 2 + kList + at, x);
            }
          }
          if (first < 0 && mask) first = cb + __ffsll((long long)mask) - 1;
          total += __popcll(mask);
        };
  #pragma unroll
        for (int t = 0; t < kScan; ++t)
          if (t * kWave < m) chunk(t * kWave, nv[t]);
        for (int cb = kScan * kWave; cb < m; cb += kWave)
          chunk(cb, cb + lane < m ? nrm2[cb + lane] : R(-1));
        int C = INT_MAX;
        const R* PVl = nullptr;        // pivot column in LDS (one workgroup) ...
        const double* PVg = nullptr;   // ... or in the exchange buffer
        if (G == 1) {
          if (Mg < R(0)) go = 0;   // every column used up
          else {
            C = c0 + first;
            PVl = colp(first);
          }
        } else {
          if (lane == 0) {
            xst(Xg, Mg);
            xst(Xg + 1, (double)total);
          }
          if (first >= 0) {
            double* Pg = PVs + (int64_t)g * (a + 1);
            if (lane == 0) xst(Pg, nrm2[first]);
            const R* fc = colp(first);
            for (int i = j + lane; i < a; i += kWave) xst(Pg + 1 + (i - j), fc[i]);
          }
          // the flag word carries the local maximum (as float) and the first
          // candidate's column, which decide the pivot whenever one group's
          // maximum exceeds all others by more than float rounding and the band
          const unsigned long long pay =
              ((unsigned long long)(first >= 0 ? c0 + first : 0xFFFF) << 32) |
              __float_as_uint((float)Mg);
          if (!wave_barrier(flags, ++phase, pay, G, g, err, &bw)) go = -1;
          bool fast = false;
          if (go > 0 && cd.list_cap == kCoopList) {
            const float Mf = lane < G ? __uint_as_float((unsigned)(bw & 0xFFFFFFFFull)) : -INFINITY;
            const float Mmax = wave_max_f(Mf);
            const unsigned long long at = __ballot(lane < G && Mf == Mmax);
            const int og = __ffsll((long long)at) - 1;
            // no other group's maximum within float rounding of og's
            const bool close = __ballot(lane < G && lane != og &&
                                        !(Mf < Mmax * (1.0f - 1.0f / (1 << 20)))) != 0ULL;
            if (Mmax < 0.0f) {
              fast = true;
              go = 0;   // every column used up
            } else if (Mmax > 0.0f && Mmax <= 3.0e38f && !close) {
              // the true maxima keep the order with a margin far above the band,
              // so the pivot is og's lowest-index candidate: its published one
              fast = true;
              C = (int)((readlane_u64(bw, og) >> 32) & 0xFFFFull);
              PVg = PVs + (int64_t)og * (a + 1);
            }
          }
          if (go > 0 && !fast) {
            // one round of loads: lane q fetches group q's maximum, count and
            // first list entry; further entries are fetched only from groups
            // that have more than one and whose maximum reaches the global band
            double Mq = -2.0, nv0 = -1.0;
            int cq = 0, ix0 = INT_MAX;
            if (lane < G) {
              const double* Xq = X + (int64_t)lane * kXs;
              Mq = xld(Xq);
              cq = (int)xld(Xq + 1);
              ix0 = (int)xld(Xq + 2);
              nv0 = xld(Xq + 2 + kList);
            }
            const double M = wave_max(Mq);
            const bool over = __ballot(lane < G && cq > cd.list_cap) != 0ULL;
            if (M < 0.0) go = 0;   // every column used up
            else {
              const double thr = M * (1.0 - PivotTie<R>::rtol);
              if (!over) {
                if (lane < G && cq > 0 && cd.list_cap > 0 && nv0 >= thr) C = ix0;
                unsigned long long more = __ballot(lane < G && cq > 1 && Mq >= thr);
                while (more) {   // rare: several candidates in one group
                  const int q = __ffsll((long long)more) - 1;
                  more &= more - 1ULL;
                  const int cqq = min(__shfl(cq, q, kWave), cd.list_cap);
                  const double* Xq = X + (int64_t)q * kXs;
                  if (lane >= 1 && lane < cqq && xld(Xq + 2 + kList + lane) >= thr)
                    C = min(C, (int)xld(Xq + 2 + lane));
                }
                C = wave_min_int(C);
              } else {
                // exact local candidates against the global threshold
                int cl = INT_MAX;
                for (int cb = 0; cb < m && cl == INT_MAX; cb += kWave) {
                  const int c = cb + lane;
                  const unsigned long long mk =
                      __ballot(c < m && nrm2[c] >= R(0) && (double)nrm2[c] >= thr);
                  if (mk) cl = c0 + cb + __ffsll((long long)mk) - 1;
                }
                if (lane == 0) xst(XB + g, (double)cl);
                if (!wave_barrier(flags, ++phase, 0, G, g, err, &bw)) go = -1;
                if (go > 0) {
                  for (int qq = lane; qq < G; qq += kWave) C = min(C, (int)xld(XB + qq));
                  C = wave_min_int(C);
                }
              }
              if (go > 0) {
                const int og = min(C / max(per, 1), G - 1);   // owner workgroup
                // the owner's published first candidate is the pivot unless the
                // lists overflowed or it fell outside the global band
                const int head_og =
                    __shfl(cq, og, kWave) > 0 && cd.list_cap > 0 ? __shfl(ix0, og, kWave) : -1;
                if (!over && head_og == C) {
                  PVg = PVs + (int64_t)og * (a + 1);
                } else {
                  if (C >= c0 && C < c1) {
                    const int Cl = C - c0;
                    if (lane == 0) xst(PVx, nrm2[Cl]);
                    const R* pc = colp(Cl);
                    for (int i = j + lane; i < a; i += kWave) xst(PVx + 1 + (i - j), pc[i]);
                  }
                  if (!wave_barrier(flags, ++phase, 0, G, g, err, &bw)) go = -1;
                  PVg = PVx;
                }
              }
            }
          }
        }
        if (go > 0) {
          // the pivot column: its norm, first entry and the next kPv * 64
          // entries are loaded together, then written to v once, scaled; the
          // entries beyond (interfaces of more than ~500 rows) go through v twice
          double pn, alpha;
          R xr[kPv];
          const int iend = min(a, j + 1 + kPv * kWave);
          if (PVl) {
            pn = nrm2[C - c0];
            alpha = PVl[j];
  #pragma unroll
            for (int t = 0; t < kPv; ++t) {
              const int i = j + 1 + lane + t * kWave;
              xr[t] = i < iend ? PVl[i] : R(0);
            }
            for (int i = iend + lane; i < a; i += kWave) v[i] = PVl[i];
          } else {
            pn = xld(PVg);
            alpha = xld(PVg + 1);
  #pragma unroll
            for (int t = 0; t < kPv; ++t) {
              const int i = j + 1 + lane + t * kWave;
              xr[t] = i < iend ? R(xld(PVg + 1 + (i - j))) : R(0);
            }
            for (int i = iend + lane; i < a; i += kWave) v[i] = R(xld(PVg + 1 + (i - j)));
          }
          const double nrm = sqrt(pn);
          if (j == 0) R00 = nrm;
          if (nrm == 0.0 || nrm < eps_stop * R00) go = 0;
          else {
            if (r < 0 && nrm < eps * R00) r = j;
            const double beta = alpha >= 0.0 ? -nrm : nrm;
            const R rden = R(1.0 / (alpha - beta));
  #pragma unroll
            for (int t = 0; t < kPv; ++t) {
              const int i = j + 1 + lane + t * kWave;
              if (i < iend) v[i] = xr[t] * rden;
            }
            for (int i = iend + lane; i < a; i += kWave) v[i] *= rden;
            if (lane == 0) {
              v[j] = 1.0;
              s_beta = beta;
              s_tau = (beta - alpha) / beta;
              sC = C;
            }
          }
        }
        if (lane == 0) {
          s_go = go;
          s_r = r;
        }
      }
      __syncthreads();
      const int go = s_go;
      if (go < 0) return;   // a group barrier timed out (error flag set)
      if (go == 0) break;
      const int C = sC;
      const R tau = R(s_tau), beta = R(s_beta);
      const bool owner = C >= c0 && C < c1;
      const int Cl = C - c0;
      if (g == 0) {
        for (int i = tid; i < a; i += kCT) d.V[i + (int64_t)j * a] = i < j ? R(0) : v[i];
        if (tid == 0) d.tau[j] = tau;
      }
      // fused reflector update + exact trailing norms; the lanes per column
      // grow as the columns per workgroup shrink, so that every wave has work
      {
        const int skip = owner ? Cl : -1;
        if (mL > kCW * 4) update_columns<8, kRpl, false>(Ys, gcol, nrm2, v, a, mL, j, tau, skip);
        else if (mL > kCW * 2)
          update_columns<16, kRpl16, false>(Ys, gcol, nrm2, v, a, mL, j, tau, skip);
        else if (mL > 0) update_columns<32, kRpl32, false>(Ys, gcol, nrm2, v, a, mL, j, tau, skip);
        if constexpr (kPanel)
          if (m > mL)
            update_columns<64, 4, true>(Ys, gcol, nrm2 + mL, v, a, m - mL, j, tau, skip - mL);
      }
      if (owner) {
        R* pc = colp(Cl);
        for (int i = j + tid; i < a; i += kCT) pc[i] = i == j ? beta : R(0);
        if (tid == 0) nrm2[Cl] = -1;
      }
      __syncthreads();
    }
    r = s_r;
    const int nref = j;
    if (r < 0) r = nref;

    // Q^T W of my columns into the transposed workspace (E^T lives in rows r..)
    for (int idx = tid; idx < m * a; idx += kCT) {
      const int c = idx % m, i = idx / m;
      d.Y[(c0 + c) + i * K] = colp(c)[i];
    }
    // coarse rows into p's panel and, transposed, into the neighbours' panels
    {
      int kk = 0;
      for (int64_t e = d.nb0; e < d.nb1; ++e) {
        const CpqrNbrT<R> nb = nbrs[e];
        const int wc = n_cur[nb.w];
        const int lo = max(kk, c0), hi = min(kk + wc, c1);
        for (int idx = tid; idx < r * (hi - lo); idx += kCT) {
          const int cc = idx % (hi - lo), i = idx / (hi - lo);
          const int cw = lo - kk + cc;  // column inside block (p, w)
          const R y = colp(lo - c0 + cc)[i];
          d.panel[i + (nb.col + cw) * a] = y;
          nb.blk_wp[cw + (int64_t)i * nb.ldw] = y;
        }
        kk += wc;
      }
    }
    if (g != 0) continue;
    for (int idx = tid; idx < r * r; idx += kCT) {
      const int i = idx % r, c = idx / r;
      d.panel[i + (d.diag_col + c) * a] = i == c ? R(1) : R(0);
    }
    if (tid == 0) {
      out_k[d.p] = k;
      out_r[d.p] = r;
      out_r2[d.p] = nref;
      n_cur[d.p] = r;
    }
  }
}

__global__ void k_fill_int(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

template <class R>
int coop_max_blocks(size_t lds_bytes, bool panel) {
  int dev = 0, ncu = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = panel ? reinterpret_cast<const void*>(k_cpqr_coop<R, true>)
                        : reinterpret_cast<const void*>(k_cpqr_coop<R, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kCT, lds_bytes) != hipSuccess)
    return 0;
  return nb * ncu;
}

void launch_fill_int(int32_t* p, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

template <class R>
hipError_t launch_cpqr_coop(const CoopDescT<R>* d, const CpqrNbrT<R>* nb, const int32_t* blk_map,
                            const int32_t* blk_ptr, int32_t nblocks, int32_t ngrid,
                            int32_t* xcd_slot, int32_t* sync, int32_t nsync, int32_t* n_cur,
                            int32_t* out_r, int32_t* out_r2, int32_t* out_k, double eps,
                            double eps_stop, int32_t* err, size_t lds_bytes, bool panel,
                            hipStream_t s) {
  if (ngrid < nblocks || ngrid % kCoopXcds != 0) return hipErrorInvalidValue;
  launch_fill_int(sync, nsync, s);
  void* args[] = {(void*)&d,        (void*)&nb,    (void*)&blk_map, (void*)&blk_ptr,
                  (void*)&nblocks,  (void*)&xcd_slot, (void*)&n_cur, (void*)&out_r,
                  (void*)&out_r2,   (void*)&out_k, (void*)&eps,     (void*)&eps_stop,
                  (void*)&err};
  const void* fn = panel ? reinterpret_cast<const void*>(k_cpqr_coop<R, true>)
                        : reinterpret_cast<const void*>(k_cpqr_coop<R, false>);
  return hipLaunchCooperativeKernel(fn, dim3(ngrid), dim3(kCT), args, lds_bytes, s);
}

template int coop_max_blocks<double>(size_t, bool);
template int coop_max_blocks<float>(size_t, bool);
template hipError_t launch_cpqr_coop<double>(const CoopDescT<double>*, const CpqrNbrT<double>*,
                                             const int32_t*, const int32_t*, int32_t, int32_t,
                                             int32_t*, int32_t*, int32_t, int32_t*, int32_t*,
                                             int32_t*, int32_t*, double, double, int32_t*, size_t,
                                             bool, hipStream_t);
template hipError_t launch_cpqr_coop<float>(const CoopDescT<float>*, const CpqrNbrT<float>*,
                                            const int32_t*, const int32_t*, int32_t, int32_t,
                                            int32_t*, int32_t*, int32_t, int32_t*, int32_t*,
                                            int32_t*, int32_t*, double, double, int32_t*, size_t,
                                            bool, hipStream_t);

}  // namespace spand
