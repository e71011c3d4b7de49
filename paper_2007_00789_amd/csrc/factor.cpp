// Host driver of the level-by-level factorization (Alg. 2).
//
// For every step l = depth ... 0 the planner lays out the row panels of the
// step's clusters (cluster c: n_c x sum_{j in adj(c)} n_j, column-major,
// both orientations of every off-diagonal block), builds flat descriptor
// lists and issues batched launches:
//   interiors : L_s^{-1} (k_potrf_inv), G_s = L_s^{-1} B_sW (k_gemm),
//               B_{w1 w2} -= G_{s,w1}^T G_{s,w2} summed over the interiors
//               bordering both, in ascending interior order (k_gemm);
//   scaling   : Z_p^{-1} (k_potrf_inv), B_pq <- Z_p^{-1} B_pq Z_q^{-T} (k_gemm x2);
//   sparsify  : one k_cpqr launch per colour;
//   merge     : parent panels assembled from the children's current blocks.
// The ranks of a step decide the next step's sizes; they are read back once
// per step (a few KB).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "runtime.h"

namespace spand {

// ---------------------------------------------------------------------------
// memory helpers
// ---------------------------------------------------------------------------
void* DevArena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (cur_ < chunks_.size()) {
    if (used_ + bytes <= chunks_[cur_].size) {
      void* p = chunks_[cur_].p + used_;
      used_ += bytes;
      return p;
    }
    ++cur_;
    used_ = 0;
  }
  size_t sz = std::max<size_t>(bytes, size_t(mirrored_ ? 16 : 64) << 20);
  Chunk c{nullptr, nullptr, sz, SIZE_MAX, 0};
  if (pool_ && pool_->take(sz, mirrored_, &c.p, &c.h, &c.size)) {
    chunks_.push_back(c);
    reserved_ += c.size;
    cur_ = chunks_.size() - 1;
    used_ = bytes;
    return c.p;
  }
  SPAND_HIP(hipMalloc(&c.p, sz));
  if (mirrored_) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c.h), sz, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipFree(c.p);
      SPAND_HIP(e);
    }
  }
  chunks_.push_back(c);
  reserved_ += sz;
  cur_ = chunks_.size() - 1;
  used_ = bytes;
  return c.p;
}

void DevArena::flush(hipStream_t s) {
  for (auto& c : chunks_)
    if (c.hi > c.lo) {
      SPAND_HIP(hipMemcpyAsync(c.p + c.lo, c.h + c.lo, c.hi - c.lo, hipMemcpyHostToDevice, s));
      c.lo = SIZE_MAX;
      c.hi = 0;
    }
}

void UploadRing::next(hipStream_t s) {
  if (!ev_[cur_]) SPAND_HIP(hipEventCreateWithFlags(&ev_[cur_], hipEventDisableTiming));
  SPAND_HIP(hipEventRecord(ev_[cur_], s));
  used_[cur_] = true;
  cur_ ^= 1;
  if (used_[cur_]) SPAND_HIP(hipEventSynchronize(ev_[cur_]));
  a_[cur_].reset();
  s_[cur_].reset();
}

UploadRing::~UploadRing() {
  for (hipEvent_t e : ev_)
    if (e) (void)hipEventDestroy(e);
}

void DevArena::mark(const char* h, size_t bytes) {
  if (bytes == 0) return;
  for (auto& c : chunks_)
    if (c.h && h >= c.h && h < c.h + c.size) {
      const size_t off = (size_t)(h - c.h);
      c.lo = std::min(c.lo, off);
      c.hi = std::max(c.hi, off + bytes);
      return;
    }
  throw Error(SPAND_E_STATE, "internal: staged descriptors outside the arena");
}

void DevArena::release() {
  for (auto& c : chunks_) {
    if (pool_) {
      pool_->give(c.p, c.h, c.size);
      continue;
    }
    (void)hipFree(c.p);
    if (c.h) (void)hipHostFree(c.h);
  }
  chunks_.clear();
  cur_ = used_ = reserved_ = 0;
}

size_t DevArena::bytes_used() const {
  size_t s = 0;
  for (size_t i = 0; i < cur_ && i < chunks_.size(); ++i) s += chunks_[i].size;
  return s + used_;
}

bool MemPool::take(size_t bytes, bool mirrored, char** dev, char** host, size_t* size) {
  std::lock_guard<std::mutex> lk(mu_);
  int best = -1;
  for (int i = 0; i < (int)idle_.size(); ++i)
    if (idle_[i].size >= bytes && (idle_[i].h != nullptr) == mirrored &&
        (best < 0 || idle_[i].size < idle_[best].size))
      best = i;
  if (best < 0) return false;
  *dev = idle_[best].d;
  *host = idle_[best].h;
  *size = idle_[best].size;
  held_ -= idle_[best].size;
  idle_.erase(idle_.begin() + best);
  return true;
}

void MemPool::give(char* dev, char* host, size_t size) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (held_ + size <= cap_) {
      idle_.push_back({dev, host, size});
      held_ += size;
      return;
    }
  }
  (void)hipSetDevice(device_);
  (void)hipFree(dev);
  if (host) (void)hipHostFree(host);
}

MemPool::~MemPool() {
  (void)hipSetDevice(device_);
  for (auto& c : idle_) {
    (void)hipFree(c.d);
    if (c.h) (void)hipHostFree(c.h);
  }
}

void* DevBuf::ensure(size_t need) {
  if (need <= bytes && p) return p;
  release();
  size_t sz = std::max<size_t>(need, 1 << 20);
  sz += sz / 4;
  char *d = nullptr, *h = nullptr;
  size_t got = 0;
  if (pool && pool->take(sz, false, &d, &h, &got)) {
    p = d;
    bytes = got;
    return p;
  }
  SPAND_HIP(hipMalloc(&p, sz));
  bytes = sz;
  return p;
}

void DevBuf::release() {
  if (p) {
    if (pool) pool->give(static_cast<char*>(p), nullptr, bytes);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

int Prof::find(const char* name) {
  for (size_t i = 0; i < entries.size(); ++i)
    if (entries[i].name == name) return (int)i;
  entries.push_back(Entry{name});
  return (int)entries.size() - 1;
}

int Prof::begin(const char* name, hipStream_t s) {
  if (!on || (!only.empty() && only != name)) return -1;
  hipEvent_t ev[2];
  for (auto& e : ev) {
    if (!pool.empty()) { e = pool.back(); pool.pop_back(); }
    else SPAND_HIP(hipEventCreate(&e));
  }
  SPAND_HIP(hipEventRecord(ev[0], s));
  pending.push_back({find(name), ev[0], ev[1]});
  return (int)pending.size() - 1;
}

void Prof::end(int id, hipStream_t s) {
  if (id < 0) return;
  SPAND_HIP(hipEventRecord(pending[id].b, s));
}

void Prof::add_work(const char* name, double w) {
  if (on && (only.empty() || only == name)) entries[find(name)].work += w;
}

void Prof::resolve() {
  for (auto& p : pending) {
    float ms = 0.f;
    SPAND_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    entries[p.entry].ms += ms;
    entries[p.entry].calls += 1;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Prof::reset() {
  entries.clear();
}

Prof::~Prof() {
  for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : pool) (void)hipEventDestroy(e);
}

Plan::~Plan() {
  if (d_rowptr) (void)hipFree(d_rowptr);
  if (d_colind) (void)hipFree(d_colind);
  if (d_leaf_dest) (void)hipFree(d_leaf_dest);
  if (d_seg_id) (void)hipFree(d_seg_id);
  if (d_seg_off) (void)hipFree(d_seg_off);
}

namespace {

inline int64_t find_adj(const StepPlan& st, int c, int target) {
  const int32_t* b = st.adj.data() + st.adj_ptr[c];
  const int32_t* e = st.adj.data() + st.adj_ptr[c + 1];
  const int32_t* it = std::lower_bound(b, e, target);
  if (it == e || *it != target) return -1;
  return st.adj_ptr[c] + (it - b);
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// output tiles (tile x tile) of an m x n GEMM (lower_only: those touching the
// lower triangle)
int64_t gemm_tile_count(int m, int n, bool lower_only, int tile) {
  const int64_t tm = ceil_div(m, tile), tn = ceil_div(n, tile);
  if (!lower_only) return tm * tn;
  int64_t c = 0;
  for (int64_t j = 0; j < tn; ++j) c += std::max<int64_t>(0, tm - j);
  return c;
}

int64_t put_gemm_tiles(TileRef* out, int32_t desc, int m, int n, bool lower_only, int tile) {
  const int tm = (int)ceil_div(m, tile), tn = (int)ceil_div(n, tile);
  int64_t c = 0;
  for (int j = 0; j < tn; ++j)
    for (int i = 0; i < tm; ++i)
      if (!lower_only || i >= j) out[c++] = TileRef{desc, i, j, 0};
  return c;
}

// Worker threads kept for the descriptor loops of the factorization (thread
// creation per loop cost more than the loops' own work at the leaf steps).
// One job at a time; a caller that finds the pool busy runs its loop alone.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool;
    return pool;
  }
  // f(i) for i in [0, count) on up to nth threads, the calling one included
  void run(int count, int nth, const std::function<void(int)>& f) {
    std::unique_lock<std::mutex> job(job_mu_, std::try_to_lock);
    if (!job.owns_lock() || nth <= 1 || count <= 1) {
      for (int i = 0; i < count; ++i) f(i);
      return;
    }
    ensure_workers(nth - 1);
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &f;
      count_ = count;
      next_.store(0);
      want_ = std::min<int>(nth - 1, (int)workers_.size());
      ++gen_;
    }
    cv_.notify_all();
    drain();
    // every index is taken: workers that have not woken yet stay out of this
    // job, those inside it are waited for
    std::unique_lock<std::mutex> lk(mu_);
    want_ = 0;
    done_cv_.wait(lk, [&] { return active_ == 0; });
    fn_ = nullptr;
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  void drain() {
    for (int i; (i = next_.fetch_add(1)) < count_;) (*fn_)(i);
  }
  void ensure_workers(int n) {
    while ((int)workers_.size() < n) workers_.emplace_back([this] { loop(); });
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_.wait(lk, [&] { return stop_ || (gen_ != seen && want_ > 0); });
      if (stop_) return;
      seen = gen_;
      --want_;
      ++active_;
      lk.unlock();
      drain();
      lk.lock();
      if (--active_ == 0) done_cv_.notify_one();
    }
  }
  std::mutex job_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> workers_;
  const std::function<void(int)>* fn_ = nullptr;
  int count_ = 0, want_ = 0, active_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

template <class Fn>
void host_parallel(int count, int nth, const Fn& f) {
  const std::function<void(int)> fn = std::cref(f);
  HostPool::get().run(count, nth, fn);
}

// threads for building a descriptor list of `items` entries on the host
int desc_threads(size_t items) {
  if (items < 16384) return 1;
  return std::min(16, (int)std::max(1u, std::thread::hardware_concurrency()));
}

void add_gemm_tiles(std::vector<TileRef>& tiles, int32_t desc, int m, int n, bool lower_only,
                    int tile) {
  const int tm = (int)ceil_div(m, tile), tn = (int)ceil_div(n, tile);
  for (int j = 0; j < tn; ++j)
    for (int i = 0; i < tm; ++i)
      if (!lower_only || i >= j) tiles.push_back({desc, i, j, 0});
}

// ---------------------------------------------------------------------------
// GEMM tile autotuning.  A GEMM launch is classed by the typical output block
// of its descriptors (the square root of their mean m n: below 96, below 192,
// below 384, above); for every class the tuner times both tile kernels (64 x 64
// and 128 x 128) on the device, on a synthetic batch of such blocks with
// k = 256 (zero operands; the timing does not depend on the values), and keeps
// the faster.  Done once per context and element type, at its first
// factorization (a few tens of milliseconds).  SPAND_GEMM_TILE=64 or 128 forces
// one kernel (measurement).
// ---------------------------------------------------------------------------
constexpr int kTuneSizes[GemmTuner::kClasses] = {64, 128, 256, 512};

int gemm_class(double mean_mn) {
  const double d = std::sqrt(std::max(mean_mn, 0.0));
  return d < 96 ? 0 : d < 192 ? 1 : d < 384 ? 2 : 3;
}

int forced_gemm_tile() {
  static const int t = [] {
    const char* e = std::getenv("SPAND_GEMM_TILE");
    const int v = e ? std::atoi(e) : 0;
    return v == kGemmTile || v == kGemmTileL ? v : 0;
  }();
  return t;
}

template <class FT>
void tune_gemm(Ctx& C) {
  const int w = sizeof(FT) == 4;
  if (C.tuner.tuned[w]) return;
  hipStream_t s = C.stream;
  // every trial launch: kTrialTiles 64 x 64 output tiles (eight per compute
  // unit) of depth kTrialK, so that both kernels run at throughput
  constexpr int K = 512;
  constexpr int64_t kTrialTiles = 2048;
  std::vector<void*> bufs;
  auto dalloc = [&](size_t bytes) {
    void* p = nullptr;
    SPAND_HIP(hipMalloc(&p, bytes));
    bufs.push_back(p);
    return p;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    SPAND_HIP(hipEventCreate(&e0));
    SPAND_HIP(hipEventCreate(&e1));
    for (int c = 0; c < GemmTuner::kClasses; ++c) {
      const int n = kTuneSizes[c];
      const int count = (int)std::max<int64_t>(1, kTrialTiles / (((int64_t)n / kGemmTile) * (n / kGemmTile)));
      FT* A = static_cast<FT*>(dalloc((size_t)K * n * sizeof(FT)));
      FT* Cm = static_cast<FT*>(dalloc((size_t)count * n * n * sizeof(FT)));
      SPAND_HIP(hipMemsetAsync(A, 0, (size_t)K * n * sizeof(FT), s));
      std::vector<GemmDescT<FT>> gd(count);
      std::vector<GemmTermT<FT>> gt(1, GemmTermT<FT>{A, A, K, K, K, 0});
      for (int i = 0; i < count; ++i) {
        GemmDescT<FT> g{};
        g.C = Cm + (size_t)i * n * n;
        g.term0 = 0;
        g.term1 = 1;
        g.ldc = n;
        g.m = n;
        g.n = n;
        g.transA = 1;
        g.alpha = -1.0;
        g.beta = 1.0;
        gd[i] = g;
      }
      auto* d_gd = static_cast<GemmDescT<FT>*>(dalloc(gd.size() * sizeof(gd[0])));
      auto* d_gt = static_cast<GemmTermT<FT>*>(dalloc(sizeof(gt[0])));
      SPAND_HIP(hipMemcpyAsync(d_gd, gd.data(), gd.size() * sizeof(gd[0]), hipMemcpyHostToDevice, s));
      SPAND_HIP(hipMemcpyAsync(d_gt, gt.data(), sizeof(gt[0]), hipMemcpyHostToDevice, s));
      float best = 0.f;
      for (int tile : {kGemmTile, kGemmTileL}) {
        std::vector<TileRef> tl;
        for (int i = 0; i < count; ++i) add_gemm_tiles(tl, i, n, n, false, tile);
        auto* d_tl = static_cast<TileRef*>(dalloc(tl.size() * sizeof(TileRef)));
        SPAND_HIP(hipMemcpyAsync(d_tl, tl.data(), tl.size() * sizeof(TileRef), hipMemcpyHostToDevice, s));
        launch_gemm(d_gd, d_gt, d_tl, (int64_t)tl.size(), kGemmNative, tile, s);   // warm-up
        std::vector<float> ms;
        for (int rep = 0; rep < 3; ++rep) {
          SPAND_HIP(hipEventRecord(e0, s));
          launch_gemm(d_gd, d_gt, d_tl, (int64_t)tl.size(), kGemmNative, tile, s);
          SPAND_HIP(hipEventRecord(e1, s));
          SPAND_HIP(hipEventSynchronize(e1));
          float t = 0.f;
          SPAND_HIP(hipEventElapsedTime(&t, e0, e1));
          ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        C.tuner.ms[w][c][tile == kGemmTileL] = ms[1];
        if (tile == kGemmTile || ms[1] < best) {
          best = ms[1];
          C.tuner.tile[w][c] = tile;
        }
      }
    }
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    for (void* p : bufs) (void)hipFree(p);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  SPAND_HIP(hipStreamSynchronize(s));
  for (void* p : bufs) (void)hipFree(p);
  C.tuner.tuned[w] = true;
}

// tile of a launch whose descriptors have this mean output size
template <class FT>
int pick_tile(const Ctx& C, const spand_opts& o, double mean_mn) {
  if (o.gemm_tile) return o.gemm_tile;
  if (const int t = forced_gemm_tile()) return t;
  return C.tuner.tile[sizeof(FT) == 4][gemm_class(mean_mn)];
}
template <class FT>
double mean_mn(const std::vector<GemmDescT<FT>>& gd) {
  double sum = 0.0;
  for (const auto& g : gd) sum += (double)g.m * g.n;
  return gd.empty() ? 0.0 : sum / (double)gd.size();
}

// Algorithmic work of a launch, recorded with the per-kernel timing: a GEMM
// launch counts 2 m n k flops per term (the lower triangle with its diagonal,
// m (m + 1) k, for a symmetric target), a Cholesky launch n^3 / 3 per block
// (the explicit inverse is not counted), a copy or fill the bytes it moves.
template <class FT>
double gemm_flops(const GemmDescT<FT>* gd, size_t ngd, const GemmTermT<FT>* gt) {
  double f = 0.0;
  for (size_t i = 0; i < ngd; ++i) {
    double k = 0.0;
    for (int64_t t = gd[i].term0; t < gd[i].term1; ++t) k += gt[t].k;
    const double mn = gd[i].lower_only ? 0.5 * gd[i].m * (gd[i].m + 1.0) : (double)gd[i].m * gd[i].n;
    f += 2.0 * mn * k;
  }
  return f;
}
template <class FT>
double gemm_flops(const std::vector<GemmDescT<FT>>& gd, const std::vector<GemmTermT<FT>>& gt) {
  return gemm_flops(gd.data(), gd.size(), gt.data());
}
template <class FT>
double potrf_flops(const std::vector<PotrfDescT<FT>>& pd) {
  double f = 0.0;
  for (const auto& p : pd) f += (double)p.n * p.n * p.n / 3.0;
  return f;
}

// One cooperative QR launch at a time per device, across every context of the
// process: a cooperative launch needs all its workgroups resident at once, and
// two of them in flight could each hold compute units the other one's waiting
// workgroups need.  Everything else of a factorization (and other contexts'
// factorizations, applies and PCG) overlaps freely with it.
std::mutex& coop_mutex(int device) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu[kMaxDevices];
  return mu[std::clamp(device, 0, kMaxDevices - 1)];
}

// the tiles of every descriptor of a launch
template <class FT>
std::vector<TileRef> tiles_of(const std::vector<GemmDescT<FT>>& gd, int tile) {
  std::vector<TileRef> tl;
  for (size_t i = 0; i < gd.size(); ++i)
    add_gemm_tiles(tl, (int32_t)i, gd[i].m, gd[i].n, gd[i].lower_only != 0, tile);
  return tl;
}

// Blocks of at most kGemmSmallN x kGemmSmallN go to the one-wave-per-block
// kernel (the leaf steps' Schur targets, which the tile kernels would pad to
// 64 x 64), unless a tile is forced (opts.gemm_tile, SPAND_GEMM_TILE) or the
// products run on the BF16 matrix cores.
bool gemm_small_ok(const spand_opts& o, GemmMode mode) {
  return mode == kGemmNative && o.gemm_tile == 0 && forced_gemm_tile() == 0;
}
bool gemm_is_small(int m, int n, bool small_ok) {
  return small_ok && m <= kGemmSmallN && n <= kGemmSmallN;
}
template <class FT>
double mean_mn_large(const std::vector<GemmDescT<FT>>& gd, bool small_ok) {
  double sum = 0.0;
  int64_t cnt = 0;
  for (const auto& g : gd)
    if (!gemm_is_small(g.m, g.n, small_ok)) {
      sum += (double)g.m * g.n;
      ++cnt;
    }
  return cnt ? sum / (double)cnt : 0.0;
}

// One GEMM launch of the factorization (native arithmetic): small blocks on
// the one-wave kernel, the others on the tile kernel chosen for their mean
// size; the algorithmic flops go to the profile of each.
template <class FT>
void run_gemm(Ctx& C, const spand_opts& o, const std::vector<GemmDescT<FT>>& gd,
              const std::vector<GemmTermT<FT>>& gt, hipStream_t s) {
  if (gd.empty()) return;
  const bool small_ok = gemm_small_ok(o, kGemmNative);
  const int tile = pick_tile<FT>(C, o, mean_mn_large(gd, small_ok));
  std::vector<TileRef> tiles, small;
  double f_small = 0.0, f_tiles = 0.0;
  const bool count = C.prof.wants("k_gemm_small") || C.prof.wants("k_gemm");
  for (size_t i = 0; i < gd.size(); ++i) {
    const GemmDescT<FT>& g = gd[i];
    const double f = count ? gemm_flops(&g, 1, gt.data()) : 0.0;
    if (gemm_is_small(g.m, g.n, small_ok)) {
      small.push_back(TileRef{(int32_t)i, 0, 0, 0});
      f_small += f;
    } else {
      add_gemm_tiles(tiles, (int32_t)i, g.m, g.n, g.lower_only != 0, tile);
      f_tiles += f;
    }
  }
  if (tiles.empty() && small.empty()) return;
  const auto* d_gd = C.upload.upload(gd);
  const auto* d_gt = C.upload.upload(gt);
  if (!small.empty()) {
    const auto* d_sm = C.upload.upload(small);
    SPAND_PROF(C, "k_gemm_small", launch_gemm_small(d_gd, d_gt, d_sm, (int64_t)small.size(), s));
    C.prof.add_work("k_gemm_small", f_small);
  }
  if (!tiles.empty()) {
    const auto* d_tl = C.upload.upload(tiles);
    SPAND_PROF(C, "k_gemm", launch_gemm(d_gd, d_gt, d_tl, (int64_t)tiles.size(), kGemmNative, tile, s));
    C.prof.add_work("k_gemm", f_tiles);
  }
}

// Blocks of at most 64 rows first, the larger ones after; the breakdown flags
// follow the same order.
template <class FT>
void order_potrf(std::vector<PotrfDescT<FT>>& pd, std::vector<int32_t>& clusters) {
  std::vector<size_t> ord(pd.size());
  std::iota(ord.begin(), ord.end(), size_t(0));
  std::stable_partition(ord.begin(), ord.end(), [&](size_t i) { return pd[i].n <= 64; });
  std::vector<PotrfDescT<FT>> p2(pd.size());
  std::vector<int32_t> c2(pd.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    p2[i] = pd[ord[i]];
    c2[i] = clusters[ord[i]];
  }
  pd.swap(p2);
  clusters.swap(c2);
}

// Many small blocks go to the one-wave-per-block kernel (its throughput is
// higher; its latency per block is not, so a few small blocks stay with the
// workgroup-per-block kernel).
constexpr int32_t kWaveBlocksMin = 2048;

template <class FT>
void launch_potrf_split(const std::vector<PotrfDescT<FT>>& pd, const PotrfDescT<FT>* d_pd,
                        int32_t* info, hipStream_t s) {
  int32_t nsmall = 0, max_s = 0, max_b = 0;
  for (const PotrfDescT<FT>& q : pd) {
    if (q.n <= 64) {
      ++nsmall;
      max_s = std::max(max_s, q.n);
    } else {
      max_b = std::max(max_b, q.n);
    }
  }
  if (nsmall < kWaveBlocksMin) {
    launch_potrf_blocks(d_pd, (int32_t)pd.size(), std::max(max_s, max_b), info, s);
    return;
  }
  launch_potrf_inv(d_pd, nsmall, max_s, info, s);
  launch_potrf_blocks(d_pd + nsmall, (int32_t)pd.size() - nsmall, max_b, info + nsmall, s);
}

// The Cholesky-inverse blocks of one launch, ready to run: the blocks factored
// in the factor's own precision and, for an FP32 factor, those factored in
// FP64 (blocks above 64 rows, and every block of the steps l <
// top_fp64_levels), each converted into an FP64 scratch copy, factored there
// and its inverse converted back.  The breakdown flags follow the order of
// `clusters`: the own blocks, then the FP64 ones.
template <class FT>
struct PotrfLaunch {
  std::vector<PotrfDescT<FT>> own;
  const PotrfDescT<FT>* d_own = nullptr;
  std::vector<PotrfDesc> wide;
  const PotrfDesc* d_wide = nullptr;
  const CopyDescT<FT, double>* d_in = nullptr;
  const CopyDescT<double, FT>* d_out = nullptr;
  std::vector<int32_t> clusters;
};

template <class FT>
void prep_potrf(Ctx& C, std::vector<PotrfDescT<FT>>& pd, std::vector<int32_t>& clusters,
                bool all_fp64, PotrfLaunch<FT>& L) {
  L = PotrfLaunch<FT>();
  if constexpr (sizeof(FT) == 8) {
    order_potrf(pd, clusters);
    L.own = std::move(pd);
    L.clusters = std::move(clusters);
    L.d_own = C.upload.upload(L.own);
  } else {
    std::vector<int32_t> cw;
    std::vector<PotrfDescT<FT>> wide_src;
    for (size_t i = 0; i < pd.size(); ++i) {
      if (all_fp64 || pd[i].n > 64) {
        wide_src.push_back(pd[i]);
        cw.push_back(clusters[i]);
      } else {
        L.own.push_back(pd[i]);
        L.clusters.push_back(clusters[i]);
      }
    }
    order_potrf(wide_src, cw);
    std::vector<CopyDescT<FT, double>> in;
    std::vector<CopyDescT<double, FT>> out;
    for (const PotrfDescT<FT>& q : wide_src) {
      const int n = q.n;
      double* A64 = C.upload.scratch_n<double>((size_t)n * n);
      double* X64 = C.upload.scratch_n<double>((size_t)n * n);
      in.push_back({q.A, A64, q.lda, n, n, n});
      L.wide.push_back({A64, X64, n, n, q.cluster, 0});
      out.push_back({X64, q.X, n, n, n, n});
    }
    L.clusters.insert(L.clusters.end(), cw.begin(), cw.end());
    L.d_own = C.upload.upload(L.own);
    L.d_wide = C.upload.upload(L.wide);
    L.d_in = C.upload.upload(in);
    L.d_out = C.upload.upload(out);
  }
}

template <class FT>
void run_potrf(const PotrfLaunch<FT>& L, int32_t* info, hipStream_t s) {
  if (!L.own.empty()) launch_potrf_split(L.own, L.d_own, info, s);
  if (!L.wide.empty()) {
    const int64_t nw = (int64_t)L.wide.size();
    launch_copy(L.d_in, nw, s);
    launch_potrf_split(L.wide, L.d_wide, info + L.own.size(), s);
    launch_copy(L.d_out, nw, s);
  }
}

void check_info(const std::vector<int32_t>& info, const std::vector<int32_t>& clusters, int l,
                const char* what) {
  for (size_t i = 0; i < info.size(); ++i)
    if (info[i] != 0)
      throw Error(SPAND_E_NOT_SPD, std::string(what) + " not SPD at step " + std::to_string(l) +
                                       ", cluster " + std::to_string(clusters[i]) + " (column " +
                                       std::to_string(info[i] - 1) + ")");
}

}  // namespace

// Position lists of step l, once its records are final: the variables of
// every cluster (the leaf vertices, or the retained variables of the children
// in step l+1, in child order) and, for a sparsified step, the columns of the
// coupling each interface was sparsified against (neighbours of earlier
// colours at their reduced sizes, in adjacency order).
void build_positions(FactorObj& F, int l) {
  const Plan& P = *F.plan;
  const StepPlan& st = P.steps[l];
  StepRec& R = F.steps[l];
  if (l == P.depth) {
    R.pos.ptr = st.vert_ptr;
    R.pos.idx = st.verts;
  } else {
    const StepPlan& ch_st = P.steps[l + 1];
    const StepRec& Rc = F.steps[l + 1];
    auto kept = [&](int ch) {
      return Rc.sparsified && ch >= ch_st.nI ? Rc.r[ch] : Rc.n0[ch];
    };
    PosLists& pos = R.pos;
    pos.ptr.assign((size_t)st.nc + 1, 0);
    pos.idx.clear();
    for (int c = 0; c < st.nc; ++c) {
      for (int64_t e = st.child_ptr[c]; e < st.child_ptr[c + 1]; ++e) {
        const int ch = st.child[e];
        pos.idx.insert(pos.idx.end(), Rc.pos.begin(ch), Rc.pos.begin(ch) + kept(ch));
      }
      pos.ptr[c + 1] = (int64_t)pos.idx.size();
      if (pos.size(c) != R.n0[c])
        throw Error(SPAND_E_STATE, "internal: cluster size mismatch at step " + std::to_string(l));
    }
  }
  R.sp_nbr_pos = PosLists{};
  if (!st.sparsified) return;
  const int nI = st.nI, nc = st.nc;
  PosLists& np = R.sp_nbr_pos;
  np.ptr.assign((size_t)nc + 1, 0);
  for (int p = nI; p < nc; ++p) {
    for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
      const int w = st.adj[e];
      if (w == p || w < nI) continue;
      const int wc = st.colour[w] < st.colour[p] ? R.r[w] : R.n0[w];
      np.idx.insert(np.idx.end(), R.pos.begin(w), R.pos.begin(w) + wc);
    }
    np.ptr[p + 1] = (int64_t)np.idx.size();
    if (np.size(p) != R.k[p])
      throw Error(SPAND_E_STATE, "internal: coupling width mismatch at step " + std::to_string(l));
  }
}

// Builds the apply program of every step whose factorization records are
// final on a host thread, beside the factorization of the later steps.
class ApplyBuilder {
 public:
  ApplyBuilder(FactorObj& F, int device) : F_(F), device_(device) {
    begin_apply(F_);
    th_ = std::thread([this] { run(); });
  }
  ApplyBuilder(const ApplyBuilder&) = delete;
  ApplyBuilder& operator=(const ApplyBuilder&) = delete;
  // steps D ... l are final
  void publish(int l) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      ready_ = l;
    }
    cv_.notify_one();
  }
  // waits for every step (all published), rethrows the builder's error
  void finish() {
    publish(0);
    th_.join();
    if (err_) std::rethrow_exception(err_);
  }
  ~ApplyBuilder() {   // error or early stop: abandon the remaining steps
    if (th_.joinable()) {
      {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
      }
      cv_.notify_one();
      th_.join();
    }
  }

 private:
  void run() {
    try {
      SPAND_HIP(hipSetDevice(device_));   // the metadata arena allocates on the factor's device
      for (int l = F_.plan->depth; l >= 0; --l) {
        {
          std::unique_lock<std::mutex> lk(mu_);
          cv_.wait(lk, [&] { return stop_ || ready_ <= l; });
          if (stop_) return;
        }
        build_positions(F_, l);
        build_apply_step(F_, l);
      }
    } catch (...) {
      err_ = std::current_exception();
    }
  }
  FactorObj& F_;
  int device_;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_;
  int ready_ = INT_MAX;
  bool stop_ = false;
  std::exception_ptr err_;
};

// Spare compute units in a cooperative QR launch: widen every group by the
// largest common factor that keeps all groups in one launch (worst-fit on the
// 8 XCDs, kCoopMaxGroup workgroups each), so that each workgroup holds fewer
// columns and its update per pivot step is shorter.  The pivot sequence does
// not depend on the group size.
template <class FT>
void widen_groups(std::vector<CoopDescT<FT>>& list) {
  auto widened = [&](double f) {
    std::vector<int> G(list.size());
    for (size_t i = 0; i < list.size(); ++i)
      G[i] = (int)std::max<int64_t>(
          list[i].G, std::min<int64_t>({(int64_t)kCoopMaxGroup, (int64_t)list[i].d.kmax,
                                        (int64_t)std::floor(list[i].G * f)}));
    return G;
  };
  auto packs = [&](const std::vector<int>& G) {
    std::vector<int> ord(G.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return G[x] > G[y]; });
    int fill[kCoopXcds] = {};
    for (int i : ord) {
      int best = -1;
      for (int x = 0; x < kCoopXcds; ++x)
        if (kCoopMaxGroup - fill[x] >= G[i] && (best < 0 || fill[x] < fill[best])) best = x;
      if (best < 0) return false;
      fill[best] += G[i];
    }
    return true;
  };
  if (list.empty() || !packs(widened(1.0))) return;
  double lo = 1.0, hi = kCoopMaxGroup;
  for (int it = 0; it < 12; ++it) {
    const double mid = 0.5 * (lo + hi);
    (packs(widened(mid)) ? lo : hi) = mid;
  }
  const std::vector<int> G = widened(lo);
  for (size_t i = 0; i < list.size(); ++i) {
    CoopDescT<FT>& q = list[i];
    if (G[i] == q.G) continue;
    const bool capped = q.ncap_lds < q.ncap;   // LDS columns limited below ncap
    const int capl = q.ncap_lds;
    q.G = G[i];
    q.ncap = (int32_t)((q.d.kmax + q.G - 1) / q.G);
    q.ncap_lds = capped ? std::min(q.ncap, capl) : q.ncap;
  }
}

namespace {

// The factorization with row panels and factor entries of type FT (double:
// SPAND_FP64; float: SPAND_FP32 and SPAND_FP32_BF16).
template <class FT>
void run_factor_t(Ctx& C, Plan& P, const double* d_vals, const spand_opts& o, FactorObj& F) {
  using PotrfD = PotrfDescT<FT>;
  using GemmD = GemmDescT<FT>;
  using GemmTm = GemmTermT<FT>;
  using CpqrD = CpqrDescT<FT>;
  using CpqrN = CpqrNbrT<FT>;
  using CoopD = CoopDescT<FT>;
  using WyD = WyDescT<FT>;
  using CopyD = CopyDescT<FT, FT>;
  auto Pt = [](void* p) { return static_cast<FT*>(p); };
  constexpr bool kF32 = sizeof(FT) == 4;
  F.f32 = kF32;
  tune_gemm<FT>(C);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = C.stream;
  const int D = P.depth;
  F.plan = &P;
  F.opts = o;
  F.steps.assign(D + 1, StepRec());
  F.arena_pool = C.pool;
  F.arena.set_pool(C.pool);
  F.meta.set_pool(C.pool);
  // the apply program is built step by step as the steps finish (not when
  // stopping after a step for a debug dump)
  std::unique_ptr<ApplyBuilder> apb;
  if (o.debug_stop_step < 0) apb = std::make_unique<ApplyBuilder>(F, C.device);
  const bool so = o.scheme == SPAND_SECOND_ORDER;
  const bool sf = o.scheme == SPAND_SUPERFINE;
  const double eps = o.eps;
  const double eps_stop = sf ? eps * eps : eps;
  double flops = 0.0;
  int64_t nnzL = 0;

  // leaf step: sizes are the vertex counts
  std::vector<int32_t> sizes(P.steps[D].nc);
  for (int c = 0; c < P.steps[D].nc; ++c)
    sizes[c] = (int32_t)(P.steps[D].vert_ptr[c + 1] - P.steps[D].vert_ptr[c]);
  // integer outputs of every step in one device buffer, the steps' regions in
  // the order D ... 0: breakdown flags of the interiors (one per interior),
  // and for a sparsified step those of the interfaces, an error word and the
  // ranks r, r2 and coupling widths k (one per cluster):
  // info_i [nI] | info_f [nc - nI] | err | r [nc] | r2 [nc] | k [nc]
  auto region = [&](int l) {
    const StepPlan& q = P.steps[l];
    return q.sparsified ? 4 * (int64_t)q.nc + 1 : std::max<int64_t>(q.nI, 1);
  };
  std::vector<int64_t> ioff(D + 1, 0);
  int64_t itotal = 0;
  for (int l = D; l >= 0; --l) {
    ioff[l] = itotal;
    itotal += (region(l) + 15) / 16 * 16;
  }
  int32_t* dint_all = static_cast<int32_t*>(C.ints.ensure(sizeof(int32_t) * itotal));
  SPAND_HIP(hipMemsetAsync(dint_all, 0, sizeof(int32_t) * itotal, s));
  // Steps without sparsification do not wait for the device: their breakdown
  // flags are read back with those of the next step that does (a failed block
  // leaves a zero inverse, so the steps in between stay finite).
  struct Deferred {
    int l;
    std::vector<int32_t> clusters;
  };
  std::vector<Deferred> deferred;
  // reads back the integer outputs of the deferred steps and of step l in one
  // copy (their regions are adjacent) and checks the breakdown flags;
  // returns step l's region
  auto read_back = [&](int l, const std::vector<int32_t>& pdc, const std::vector<int32_t>& zdc) {
    const int64_t lo = deferred.empty() ? ioff[l] : ioff[deferred.front().l];
    std::vector<int32_t> hb((size_t)(ioff[l] + region(l) - lo));
    SPAND_HIP(hipMemcpyAsync(hb.data(), dint_all + lo, sizeof(int32_t) * hb.size(),
                             hipMemcpyDeviceToHost, s));
    SPAND_HIP(hipStreamSynchronize(s));
    auto flags = [&](int ls, int64_t at, size_t count) {
      const size_t b = (size_t)(ioff[ls] - lo + at);
      return std::vector<int32_t>(hb.begin() + b, hb.begin() + b + count);
    };
    for (const Deferred& d : deferred)
      check_info(flags(d.l, 0, d.clusters.size()), d.clusters, d.l, "interior block");
    deferred.clear();
    check_info(flags(l, 0, pdc.size()), pdc, l, "interior block");
    check_info(flags(l, P.steps[l].nI, zdc.size()), zdc, l, "interface block");
    return std::vector<int32_t>(hb.begin() + (ioff[l] - lo), hb.end());
  };

  int cur = 0;
  PanelLayout lay_store;
  const PanelLayout* layp = &P.leaf_layout;
  FT* panel = static_cast<FT*>(C.panels[cur].ensure(layp->total * sizeof(FT)));
  SPAND_PROF(C, "k_fill", launch_fill(panel, layp->total, 0.0, s));
  SPAND_PROF(C, "k_scatter", launch_scatter(d_vals, P.d_leaf_dest, P.nnz, panel, s));
  C.prof.add_work("k_fill", (double)layp->total * sizeof(FT));
  C.prof.add_work("k_scatter", (double)P.nnz * (sizeof(double) + sizeof(int64_t) + sizeof(FT)));

  for (int l = D; l >= 0; --l) {
    const StepPlan& st = P.steps[l];
    StepRec& R = F.steps[l];
    const PanelLayout& lay = *layp;
    C.upload.next(s);
    R.l = l;
    R.sparsified = st.sparsified;
    R.n0 = sizes;
    const int nI = st.nI, nc = st.nc;
    R.r.assign(nc, -1);
    R.r2.assign(nc, -1);
    R.k.assign(nc, -1);
    R.Linv.assign(nc, nullptr);
    R.G.assign(nc, nullptr);
    R.kint.assign(nc, 0);
    R.Zinv.assign(nc, nullptr);
    R.Y.assign(nc, nullptr);
    R.V.assign(nc, nullptr);
    R.tau.assign(nc, nullptr);
    R.T.assign(nc, nullptr);
    R.VT.assign(nc, nullptr);
    R.kmax.assign(nc, 0);
    auto blk = [&](int c, int64_t e) { return panel + lay.off[c] + lay.coff[e] * lay.n[c]; };

    // this step's integer outputs (cleared at the start); the current sizes
    // n_cur start as a copy of the sizes in the step's upload buffer
    int32_t* dint = dint_all + ioff[l];
    int32_t* d_info_i = dint;
    int32_t* d_info_f = st.sparsified ? dint + nI : nullptr;
    int32_t* d_err = st.sparsified ? dint + nc : nullptr;
    int32_t* d_r = st.sparsified ? dint + nc + 1 : nullptr;
    int32_t* d_r2 = st.sparsified ? d_r + nc : nullptr;
    int32_t* d_k = st.sparsified ? d_r + 2 * nc : nullptr;
    int32_t* d_ncur = C.upload.upload(sizes);

    // ---------------- (a) interiors ----------------
    std::vector<PotrfD> pd;
    std::vector<int32_t> pd_cluster;
    int max_n = 0;
    for (int sI = 0; sI < nI; ++sI) {
      const int ns = sizes[sI];
      const int64_t ks = lay.width[sI] - ns;
      R.kint[sI] = (int32_t)ks;
      if (ns == 0) continue;
      R.Linv[sI] = F.arena.alloc_n<FT>((size_t)ns * ns);
      if (ks > 0) R.G[sI] = F.arena.alloc_n<FT>((size_t)ns * ks);
      pd.push_back({panel + lay.off[sI], Pt(R.Linv[sI]), ns, ns, sI, 0});
      pd_cluster.push_back(sI);
      max_n = std::max(max_n, ns);
      flops += (double)ns * ns * ns / 3.0 + (double)ns * ns * ks + (double)ns * ks * ks;
      nnzL += (int64_t)ns * (ns + 1) / 2 + (int64_t)ns * ks;
    }
    if (max_n > 3500) throw Error(SPAND_E_LIMIT, "interior block larger than 3500");
    if (!pd.empty()) {
      PotrfLaunch<FT> pl;
      const double pd_flops = C.prof.wants("k_potrf_inv") ? potrf_flops(pd) : 0.0;
      prep_potrf(C, pd, pd_cluster, l < o.top_fp64_levels, pl);
      pd_cluster = pl.clusters;
      SPAND_PROF(C, "k_potrf_inv", run_potrf(pl, d_info_i, s));
      C.prof.add_work("k_potrf_inv", pd_flops);
      // G_s = L_s^{-1} B_{s,W}
      std::vector<GemmD> gd;
      std::vector<GemmTm> gt;
      for (int sI = 0; sI < nI; ++sI) {
        const int ns = sizes[sI];
        const int ks = R.kint[sI];
        if (ns == 0 || ks == 0) continue;
        gt.push_back({Pt(R.Linv[sI]), panel + lay.off[sI] + (int64_t)ns * ns, ns, ns, ns, 0});
        GemmD g{};
        g.C = Pt(R.G[sI]);
        g.C2 = nullptr;
        g.term0 = (int64_t)gt.size() - 1;
        g.term1 = (int64_t)gt.size();
        g.ldc = ns;
        g.m = ns;
        g.n = ks;
        g.alpha = 1.0;
        g.beta = 0.0;
        gd.push_back(g);
      }
      run_gemm(C, o, gd, gt, s);
      // Schur complement: B_{w1 w2} -= sum_s G_{s,w1}^T G_{s,w2} (structure
      // from the plan: targets and their interiors in ascending order).  The
      // descriptors are written in place into the pinned upload buffer, in
      // chunks of targets on several threads for large steps: a counting pass
      // gives every chunk its offsets, a second pass writes.
      const int64_t nsch = (int64_t)st.schur.size();
      const int nth = desc_threads((size_t)nsch);
      const int nchunk = nth > 1 ? 4 * nth : 1;
      std::vector<int64_t> o_gd(nchunk + 1, 0), o_gt(nchunk + 1, 0), o_tl(nchunk + 1, 0),
          o_sm(nchunk + 1, 0);
      // the Schur products from BF16 operands below the top FP64 levels
      // (SPAND_FP32_BF16); in the panels' own precision otherwise
      const GemmMode sm = o.precision == SPAND_FP32_BF16 && l >= o.top_fp64_levels ? kGemmBf16
                                                                                   : kGemmNative;
      const bool small_ok = gemm_small_ok(o, sm);
      auto live_terms = [&](const StepPlan::SchurTarget& tg) {
        int64_t t = 0;
        for (int64_t q = tg.t0; q < tg.t1; ++q) t += sizes[st.schur_terms[q].s] != 0;
        return t;
      };
      // tile of the launch from the mean size of its live target blocks
      // (those that the tile kernel takes)
      double sch_mn = 0.0;
      int64_t sch_n = 0;
      for (const StepPlan::SchurTarget& tg : st.schur)
        if (sizes[tg.w1] != 0 && sizes[tg.w2] != 0 &&
            !gemm_is_small(sizes[tg.w1], sizes[tg.w2], small_ok)) {
          sch_mn += (double)sizes[tg.w1] * sizes[tg.w2];
          ++sch_n;
        }
      const int stile = pick_tile<FT>(C, o, sch_n ? sch_mn / (double)sch_n : 0.0);
      host_parallel(nchunk, nth, [&](int c) {
        int64_t ngd = 0, ngt = 0, ntl = 0, nsm = 0;
        for (int64_t i = nsch * c / nchunk; i < nsch * (c + 1) / nchunk; ++i) {
          const StepPlan::SchurTarget& tg = st.schur[i];
          if (sizes[tg.w1] == 0 || sizes[tg.w2] == 0) continue;
          const int64_t t = live_terms(tg);
          if (t == 0) continue;
          ++ngd;
          ngt += t;
          if (gemm_is_small(sizes[tg.w1], sizes[tg.w2], small_ok)) ++nsm;
          else ntl += gemm_tile_count(sizes[tg.w1], sizes[tg.w2], tg.w1 == tg.w2, stile);
        }
        o_gd[c + 1] = ngd;
        o_gt[c + 1] = ngt;
        o_tl[c + 1] = ntl;
        o_sm[c + 1] = nsm;
      });
      for (int c = 0; c < nchunk; ++c) {
        o_gd[c + 1] += o_gd[c];
        o_gt[c + 1] += o_gt[c];
        o_tl[c + 1] += o_tl[c];
        o_sm[c + 1] += o_sm[c];
      }
      if (o_tl[nchunk] + o_sm[nchunk] > 0) {
        GemmD* d_sgd = nullptr;
        GemmTm* d_sgt = nullptr;
        TileRef* d_stl = nullptr;
        TileRef* d_ssm = nullptr;
        GemmD* hgd = C.upload.stage<GemmD>((size_t)o_gd[nchunk], &d_sgd);
        GemmTm* hgt = C.upload.stage<GemmTm>((size_t)o_gt[nchunk], &d_sgt);
        TileRef* htl = C.upload.stage<TileRef>((size_t)std::max<int64_t>(o_tl[nchunk], 1), &d_stl);
        TileRef* hsm = C.upload.stage<TileRef>((size_t)std::max<int64_t>(o_sm[nchunk], 1), &d_ssm);
        host_parallel(nchunk, nth, [&](int c) {
          int64_t igd = o_gd[c], igt = o_gt[c], itl = o_tl[c], ism = o_sm[c];
          for (int64_t i = nsch * c / nchunk; i < nsch * (c + 1) / nchunk; ++i) {
            const StepPlan::SchurTarget& tg = st.schur[i];
            const int w1 = tg.w1, w2 = tg.w2;
            if (sizes[w1] == 0 || sizes[w2] == 0) continue;
            const int64_t t0 = igt;
            for (int64_t q = tg.t0; q < tg.t1; ++q) {
              const StepPlan::SchurTerm& tm = st.schur_terms[q];
              const int ns = sizes[tm.s];
              if (ns == 0) continue;
              const int64_t c1 = lay.coff[tm.e1] - ns;
              const int64_t c2 = lay.coff[tm.e2] - ns;
              hgt[igt++] = GemmTm{Pt(R.G[tm.s]) + c1 * ns, Pt(R.G[tm.s]) + c2 * ns, ns, ns, ns, 0};
            }
            if (igt == t0) continue;
            GemmD& g = hgd[igd];
            g = GemmD{};
            g.C = blk(w1, tg.e);
            g.C2 = w1 == w2 ? nullptr : blk(w2, st.adj_rev[tg.e]);
            g.term0 = t0;
            g.term1 = igt;
            g.ldc = sizes[w1];
            g.ldc2 = sizes[w2];
            g.m = sizes[w1];
            g.n = sizes[w2];
            g.transA = 1;
            g.transB = 0;
            g.lower_only = w1 == w2;
            g.alpha = -1.0;
            g.beta = 1.0;
            if (gemm_is_small(g.m, g.n, small_ok)) hsm[ism++] = TileRef{(int32_t)igd, 0, 0, 0};
            else itl += put_gemm_tiles(htl + itl, (int32_t)igd, g.m, g.n, w1 == w2, stile);
            ++igd;
          }
        });
        double f_small = 0.0, f_all = 0.0;
        if (C.prof.wants("k_gemm_small") || C.prof.wants("k_gemm")) {
          f_all = gemm_flops(hgd, (size_t)o_gd[nchunk], hgt);
          for (int64_t i = 0; i < o_sm[nchunk]; ++i) f_small += gemm_flops(hgd + hsm[i].desc, 1, hgt);
        }
        C.upload.commit(hgd, (size_t)o_gd[nchunk]);
        C.upload.commit(hgt, (size_t)o_gt[nchunk]);
        C.upload.commit(htl, (size_t)std::max<int64_t>(o_tl[nchunk], 1));
        C.upload.commit(hsm, (size_t)std::max<int64_t>(o_sm[nchunk], 1));
        if (o_sm[nchunk] > 0) {
          SPAND_PROF(C, "k_gemm_small", launch_gemm_small(d_sgd, d_sgt, d_ssm, o_sm[nchunk], s));
          C.prof.add_work("k_gemm_small", f_small);
        }
        if (o_tl[nchunk] > 0) {
          SPAND_PROF(C, "k_gemm", launch_gemm(d_sgd, d_sgt, d_stl, o_tl[nchunk], sm, stile, s));
          C.prof.add_work("k_gemm", f_all - f_small);
        }
      }
    }

    if (l == 0) {
      read_back(l, pd_cluster, {});
      F.stats.root_size = nc > 0 ? sizes[0] : 0;
      break;
    }

    // ---------------- (b) scaling and (c) sparsification ----------------
    std::vector<char> coop_used;
    // held from the step's first cooperative QR launch until its ranks are
    // read back (the device has finished them)
    std::unique_lock<std::mutex> coop_lk(coop_mutex(C.device), std::defer_lock);
    std::vector<PotrfD> zd;
    std::vector<int32_t> zd_cluster;
    if (st.sparsified) {
      int max_a = 0;
      for (int p = nI; p < nc; ++p) {
        const int a = sizes[p];
        if (a == 0) continue;
        R.Zinv[p] = F.arena.alloc_n<FT>((size_t)a * a);
        zd.push_back({blk(p, find_adj(st, p, p)), Pt(R.Zinv[p]), a, a, p, 0});
        zd_cluster.push_back(p);
        max_a = std::max(max_a, a);
        flops += (double)a * a * a / 3.0;
        nnzL += (int64_t)a * (a + 1) / 2;
      }
      if (max_a > 3500) throw Error(SPAND_E_LIMIT, "interface block larger than 3500");
      PotrfLaunch<FT> zl;
      const double zd_flops = C.prof.wants("k_potrf_inv") ? potrf_flops(zd) : 0.0;
      prep_potrf(C, zd, zd_cluster, l < o.top_fp64_levels, zl);
      zd_cluster = zl.clusters;
      SPAND_PROF(C, "k_potrf_inv", run_potrf(zl, d_info_f, s));
      C.prof.add_work("k_potrf_inv", zd_flops);
      // two-sided scaling of every interface pair p < q
      std::vector<GemmD> g1, g2;
      std::vector<GemmTm> t1, t2;
      int64_t toff = 0;
      std::vector<int64_t> tpos;
      for (int p = nI; p < nc; ++p)
        for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
          const int q = st.adj[e];
          if (q <= p || sizes[p] == 0 || sizes[q] == 0) continue;
          tpos.push_back(toff);
          toff += (int64_t)sizes[p] * sizes[q];
        }
      FT* T = static_cast<FT*>(C.temp.ensure(std::max<int64_t>(toff, 1) * sizeof(FT)));
      size_t ti = 0;
      for (int p = nI; p < nc; ++p)
        for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
          const int q = st.adj[e];
          if (q <= p || sizes[p] == 0 || sizes[q] == 0) continue;
          const int ap = sizes[p], aq = sizes[q];
          FT* Tpq = T + tpos[ti++];
          t1.push_back({Pt(R.Zinv[p]), blk(p, e), ap, ap, ap, 0});
          GemmD a{};
          a.C = Tpq;
          a.term0 = (int64_t)t1.size() - 1;
          a.term1 = (int64_t)t1.size();
          a.ldc = ap;
          a.m = ap;
          a.n = aq;
          a.alpha = 1.0;
          g1.push_back(a);
          t2.push_back({Tpq, Pt(R.Zinv[q]), ap, aq, aq, 0});
          GemmD b{};
          b.C = blk(p, e);
          b.C2 = blk(q, st.adj_rev[e]);
          b.term0 = (int64_t)t2.size() - 1;
          b.term1 = (int64_t)t2.size();
          b.ldc = ap;
          b.ldc2 = aq;
          b.m = ap;
          b.n = aq;
          b.transB = 1;
          b.alpha = 1.0;
          g2.push_back(b);
        }
      run_gemm(C, o, g1, t1, s);
      run_gemm(C, o, g2, t2, s);
      // sparsification, one launch per colour: interfaces whose coupling fits
      // in the LDS of at most kCoopMaxGroup workgroups run the cooperative QR,
      // the others the single-workgroup QR on a global-memory workspace
      coop_used.assign(nc, 0);
      coop_lk.lock();
      // The barrier words of every cooperative group of the step (at most one
      // group per interface) are cleared by one fill before the first launch;
      // each colour is launched as soon as it is planned.
      // after them, the 8 XCD slot counters of every launch (at most one
      // launch per interface), cleared by the same fill
      const int64_t sync_cap = (int64_t)std::max(nc - nI, 1) * kCoopSyncInts;
      const int64_t xcd_cap = (int64_t)std::max(nc - nI, 1) * kCoopXcds;
      int32_t* sync_all = C.upload.scratch_n<int32_t>((size_t)(sync_cap + xcd_cap));
      launch_fill_int(sync_all, sync_cap + xcd_cap, s);
      int64_t sync_used = 0, xcd_used = 0;
      for (int colour = 0; colour < st.ncolours; ++colour) {
        std::vector<CpqrD> cd;
        std::vector<CoopD> qd;
        std::vector<CpqrN> cn;
        int ma = 1, mk = 1;
        for (int p : st.order) {
          if (st.colour[p] != colour) continue;
          const int a = sizes[p];
          CpqrD d{};
          d.panel = panel + lay.off[p];
          d.a = a;
          d.p = p;
          d.nb0 = (int64_t)cn.size();
          int64_t kmax = 0;
          for (int64_t e = st.adj_ptr[p]; e < st.adj_ptr[p + 1]; ++e) {
            const int w = st.adj[e];
            if (w == p) { d.diag_col = lay.coff[e]; continue; }
            if (w < nI) continue;
            CpqrN nb{};
            nb.blk_wp = blk(w, st.adj_rev[e]);
            nb.col = lay.coff[e];
            nb.w = w;
            nb.ldw = sizes[w];
            cn.push_back(nb);
            kmax += sizes[w];
          }
          d.nb1 = (int64_t)cn.size();
          d.kmax = (int32_t)kmax;
          R.kmax[p] = kmax;
          const int64_t mn = std::min<int64_t>(a, kmax);
          if (a > 0 && kmax > 0) {
            R.Y[p] = F.arena.alloc_n<FT>((size_t)a * kmax);
            R.V[p] = F.arena.alloc_n<FT>((size_t)a * mn);
            R.tau[p] = F.arena.alloc_n<FT>((size_t)mn);
            R.T[p] = F.arena.alloc_n<FT>((size_t)mn * mn);
          }
          d.Y = Pt(R.Y[p]);
          d.V = Pt(R.V[p]);
          d.tau = Pt(R.tau[p]);
          d.T = Pt(R.T[p]);
          const int64_t cap = !(a > 0) ? 0 : coop_cols<FT>(a);
          int64_t G = cap > 0 ? (kmax + cap - 1) / cap : 0;
          if (o.qr_group > 0) G = std::max(G, std::min<int64_t>(o.qr_group, kmax));
          // too wide for kCoopMaxGroup workgroups' LDS: kCoopMaxGroup
          // workgroups, each keeping its columns beyond the LDS in the panel
          if (G > kCoopMaxGroup && o.qr_group >= 0 &&
              (kmax + kCoopMaxGroup - 1) / kCoopMaxGroup <= kCoopOverflow * cap)
            G = kCoopMaxGroup;
          if (o.qr_group >= 0 && a > 0 && kmax > 0 && G >= 1 && G <= kCoopMaxGroup) {
            CoopD q{};
            q.d = d;
            q.G = (int32_t)G;
            q.ncap = (int32_t)((kmax + G - 1) / G);
            int64_t capl = cap;
            if (o.qr_lds_cols > 0) capl = std::min<int64_t>(capl, o.qr_lds_cols);
            q.ncap_lds = (int32_t)std::min<int64_t>(q.ncap, capl);
            q.list_cap = o.qr_list_cap < 0 ? 32 : o.qr_list_cap;
            qd.push_back(q);
            coop_used[p] = 1;
            continue;
          }
          if (kmax > kCpqrMaxK) throw Error(SPAND_E_LIMIT, "interface coupling wider than " +
                                                               std::to_string(kCpqrMaxK));
          ma = std::max(ma, a);
          mk = std::max<int>(mk, (int)kmax);
          cd.push_back(d);
        }
        const CpqrN* d_cn = C.upload.upload(cn);
        if (!cd.empty()) {
          const auto* d_cd = C.upload.upload(cd);
          SPAND_PROF(C, "k_cpqr", launch_cpqr(d_cd, d_cn, (int32_t)cd.size(), d_ncur, d_r, d_r2,
                                              d_k, eps, eps_stop, ma, mk, s));
        }
        // cooperative groups, packed onto XCDs (all workgroups of a group on
        // one XCD; block b of a launch runs on XCD b % kCoopXcds) in rounds of
        // as many groups as can be co-resident.  The rounds of a colour run
        // as one launch (each workgroup takes its next group as soon as its
        // previous one is done, no launch boundary between rounds), or
        // (opts.qr_single_launch = 0) as one launch each.
        {
          std::vector<CoopD>& list = qd;
          size_t lds = 0;
          int cap_blocks = 0;
          bool panel = false;   // some workgroup keeps columns in the row panel
          for (const CoopD& q : list) panel = panel || q.ncap_lds < q.ncap;
          for (const CoopD& q : list)
            lds = std::max(lds, coop_lds_bytes<FT>(q.d.a, q.ncap, q.ncap_lds));
          if (!list.empty()) cap_blocks = coop_max_blocks<FT>(lds, panel);
          const int slots = cap_blocks / kCoopXcds;
          if (!list.empty() && slots <= 0)
            throw Error(SPAND_E_HIP, "cooperative QR cannot be made resident");
          std::vector<int> ord(list.size());
          for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
          std::stable_sort(ord.begin(), ord.end(),
                           [&](int x, int y) { return list[x].G > list[y].G; });
          std::vector<char> done(list.size(), 0);
          size_t ndone = 0;
          struct Round {
            std::vector<CoopD> q;
            std::vector<int> xcd, slot;
            int maxfill;
          };
          std::vector<Round> rounds;
          while (ndone < list.size()) {
            int fill[kCoopXcds] = {};
            std::vector<int> members, at_xcd, at_slot;
            for (int i : ord) {
              if (done[i]) continue;
              const int G = list[i].G;
              if (G > slots) throw Error(SPAND_E_LIMIT, "cooperative QR group larger than an XCD");
              int best = -1;
              for (int x = 0; x < kCoopXcds; ++x)
                if (slots - fill[x] >= G && (best < 0 || fill[x] < fill[best])) best = x;
              if (best < 0) continue;   // goes to the next launch
              members.push_back(i);
              at_xcd.push_back(best);
              at_slot.push_back(fill[best]);
              fill[best] += G;
              done[i] = 1;
              ++ndone;
            }
            // compute units this launch leaves idle: widen its groups and
            // place them again (the pivot sequence does not depend on G)
            std::vector<CoopD> mq;
            for (int i : members) mq.push_back(list[i]);
            if (o.qr_group == 0 && slots >= kCoopMaxGroup) {
              std::vector<CoopD> wq = mq;
              widen_groups(wq);
              bool changed = false;
              for (size_t b = 0; b < wq.size(); ++b) changed = changed || wq[b].G != mq[b].G;
              if (changed) {
                std::vector<int> om(wq.size());
                std::iota(om.begin(), om.end(), 0);
                std::stable_sort(om.begin(), om.end(), [&](int x, int y) { return wq[x].G > wq[y].G; });
                int f2[kCoopXcds] = {};
                std::vector<int> ax(wq.size()), as(wq.size());
                bool ok = true;
                for (int b : om) {
                  int best = -1;
                  for (int x = 0; x < kCoopXcds; ++x)
                    if (slots - f2[x] >= wq[b].G && (best < 0 || f2[x] < f2[best])) best = x;
                  if (best < 0) {
                    ok = false;
                    break;
                  }
                  ax[b] = best;
                  as[b] = f2[best];
                  f2[best] += wq[b].G;
                }
                if (ok) {
                  mq = wq;
                  at_xcd = ax;
                  at_slot = as;
                  std::copy(f2, f2 + kCoopXcds, fill);
                }
              }
            }
            rounds.push_back({std::move(mq), std::move(at_xcd), std::move(at_slot),
                              *std::max_element(fill, fill + kCoopXcds)});
          }
          // rounds [r0, r1) in one launch: block b's memberships in round
          // order, so that a group waits only for groups of earlier rounds
          auto launch_rounds = [&](size_t r0, size_t r1) {
            int maxfill = 0;
            int64_t xdoubles = 0, ngroups = 0;
            for (size_t r = r0; r < r1; ++r) {
              maxfill = std::max(maxfill, rounds[r].maxfill);
              for (const CoopD& q : rounds[r].q) xdoubles += coop_xch_doubles(q.G, q.d.a);
              ngroups += (int64_t)rounds[r].q.size();
            }
            const int nblocks = maxfill * kCoopXcds;
            int32_t* sync = sync_all + sync_used;
            sync_used += ngroups * kCoopSyncInts;
            if (sync_used > sync_cap)
              throw Error(SPAND_E_STATE, "internal: cooperative QR barrier words exhausted");
            double* xch = C.upload.scratch_n<double>((size_t)xdoubles);
            std::vector<CoopD> batch;
            batch.reserve((size_t)ngroups);
            std::vector<std::vector<int32_t>> member_of((size_t)nblocks);
            int64_t xo = 0;
            for (size_t r = r0; r < r1; ++r) {
              const Round& rd = rounds[r];
              for (size_t bi = 0; bi < rd.q.size(); ++bi) {
                CoopD q = rd.q[bi];
                const int64_t gi = (int64_t)batch.size();
                q.xcd = o.qr_xcd_local ? rd.xcd[bi] : -1;
                q.sync = sync + gi * kCoopSyncInts;
                q.xch = xch + xo;
                xo += coop_xch_doubles(q.G, q.d.a);
                for (int g = 0; g < q.G; ++g)
                  member_of[rd.xcd[bi] + (size_t)kCoopXcds * (rd.slot[bi] + g)].push_back(
                      (int32_t)(gi * kCoopMaxGroup + g));
                batch.push_back(q);
              }
            }
            const int32_t* d_map = nullptr;
            const int32_t* d_ptr = nullptr;
            if (r1 - r0 == 1) {
              std::vector<int32_t> blk_map((size_t)nblocks, -1);
              for (int b = 0; b < nblocks; ++b)
                if (!member_of[b].empty()) blk_map[b] = member_of[b][0];
              d_map = C.upload.upload(blk_map);
            } else {
              // [block pointers (nblocks + 1) | memberships]
              std::vector<int32_t> lists((size_t)nblocks + 1);
              for (int b = 0; b < nblocks; ++b) {
                lists[b] = (int32_t)(lists.size() - (size_t)nblocks - 1);
                lists.insert(lists.end(), member_of[b].begin(), member_of[b].end());
              }
              lists[nblocks] = (int32_t)(lists.size() - (size_t)nblocks - 1);
              d_ptr = C.upload.upload(lists);
              d_map = d_ptr + nblocks + 1;
            }
            const auto* d_qd = C.upload.upload(batch);
            int32_t* d_xs = sync_all + sync_cap + xcd_used;
            xcd_used += kCoopXcds;
            if (xcd_used > xcd_cap)
              throw Error(SPAND_E_STATE, "internal: cooperative QR slot counters exhausted");
            hipError_t he = hipSuccess;
            SPAND_PROF(C, "k_cpqr_coop",
                       he = launch_cpqr_coop(d_qd, d_cn, d_map, d_ptr, nblocks,
                                             slots * kCoopXcds, d_xs, nullptr, 0, d_ncur, d_r,
                                             d_r2, d_k, eps, eps_stop, d_err, lds, panel, s));
            SPAND_HIP(he);
          };
          if (o.qr_single_launch && !rounds.empty()) launch_rounds(0, rounds.size());
          else
            for (size_t r = 0; r < rounds.size(); ++r) launch_rounds(r, r + 1);
        }
      }
    }
    // ranks and breakdown flags: read back at sparsified steps (and when
    // stopping after this step), deferred otherwise
    const bool stop_here = o.debug_stop_step == l;
    std::vector<int32_t> cur_sizes = sizes;  // sizes after this step's sparsification
    if (st.sparsified || stop_here) {
      const std::vector<int32_t> hb = read_back(l, pd_cluster, zd_cluster);
      if (coop_lk.owns_lock()) coop_lk.unlock();
      if (st.sparsified) {
        const int32_t herr = hb[nc];
        if (herr & 1) throw Error(SPAND_E_STATE, "cooperative QR timed out at step " + std::to_string(l));
        if (herr & 2) throw CoopPlacement();
        for (int p = nI; p < nc; ++p) {
          R.r[p] = hb[(size_t)nc + 1 + p];
          R.r2[p] = hb[2 * (size_t)nc + 1 + p];
          R.k[p] = hb[3 * (size_t)nc + 1 + p];
          cur_sizes[p] = R.r[p];
        }
      }
    } else {
      deferred.push_back({l, std::move(pd_cluster)});
    }

    // ---------------- (d) merge into step l-1 ----------------
    // launched as soon as the ranks are known; the host bookkeeping of this
    // step (positions, statistics, apply records) follows while it runs
    std::vector<int32_t> nsz;
    PanelLayout nlay;
    FT* npanel = nullptr;
    if (!stop_here) {
      const StepPlan& nx = P.steps[l - 1];
      nsz.assign(nx.nc, 0);
      std::vector<int32_t> choff(st.nc, 0);  // row offset of a child inside its parent
      for (int c = 0; c < nx.nc; ++c)
        for (int64_t e = nx.child_ptr[c]; e < nx.child_ptr[c + 1]; ++e) {
          const int ch = nx.child[e];
          choff[ch] = nsz[c];
          nsz[c] += cur_sizes[ch];
        }
      nlay = make_layout(nx, nsz);
      npanel = static_cast<FT*>(
          C.panels[1 - cur].ensure(std::max<int64_t>(nlay.total, 1) * sizeof(FT)));
      SPAND_PROF(C, "k_fill", launch_fill(npanel, nlay.total, 0.0, s));
      C.prof.add_work("k_fill", (double)nlay.total * sizeof(FT));
      const int64_t nm = (int64_t)st.merge.size();
      const int mth = desc_threads((size_t)nm);
      const int mchunk = mth > 1 ? 4 * mth : 1;
      std::vector<int64_t> o_cp(mchunk + 1, 0);
      auto live = [&](const StepPlan::MergeCopy& mc) {
        return cur_sizes[mc.ci] != 0 && cur_sizes[mc.cj] != 0;
      };
      host_parallel(mchunk, mth, [&](int c) {
        int64_t k = 0;
        for (int64_t i = nm * c / mchunk; i < nm * (c + 1) / mchunk; ++i) k += live(st.merge[i]);
        o_cp[c + 1] = k;
      });
      for (int c = 0; c < mchunk; ++c) o_cp[c + 1] += o_cp[c];
      CopyD* d_cp = nullptr;
      CopyD* hcp = C.upload.stage<CopyD>((size_t)o_cp[mchunk], &d_cp);
      host_parallel(mchunk, mth, [&](int c) {
        int64_t k = o_cp[c];
        for (int64_t i = nm * c / mchunk; i < nm * (c + 1) / mchunk; ++i) {
          const StepPlan::MergeCopy& mc = st.merge[i];
          if (!live(mc)) continue;
          const int ci = mc.ci, cj = mc.cj, P_ = mc.P;
          CopyD& d = hcp[k++];
          d.src = blk(ci, mc.ee);
          d.lds = sizes[ci];
          d.dst = npanel + nlay.off[P_] + (nlay.coff[mc.e] + choff[cj]) * nsz[P_] + choff[ci];
          d.ldd = nsz[P_];
          d.m = cur_sizes[ci];
          d.n = cur_sizes[cj];
        }
      });
      if (C.prof.wants("k_copy")) {
        double bytes = 0.0;
        for (int64_t i = 0; i < o_cp[mchunk]; ++i) bytes += 2.0 * hcp[i].m * hcp[i].n * sizeof(FT);
        C.prof.add_work("k_copy", bytes);
      }
      C.upload.commit(hcp, (size_t)o_cp[mchunk]);
      SPAND_PROF(C, "k_copy", launch_copy(d_cp, o_cp[mchunk], s));
    }

    if (st.sparsified) {
      // statistics, and room for V T (formed at the end); the position lists
      // of this step are built by the apply builder
      for (int p = nI; p < nc; ++p) {
        const int a = sizes[p], r = R.r[p], r2 = R.r2[p], k = R.k[p];
        if (Pt(R.V[p]) && r2 > 0) R.VT[p] = F.arena.alloc_n<FT>((size_t)a * r2);   // V T, formed at the end
        flops += (double)a * a * k;
        double qr = 0.0;
        for (int j = 0; j < r2; ++j) qr += 4.0 * (a - j) * (double)(k - j);
        flops += qr;
        C.prof.add_work(coop_used[p] ? "k_cpqr_coop" : "k_cpqr", qr);
        nnzL += (int64_t)a * r2 - (int64_t)r2 * (r2 - 1) / 2 + r2;
        if (so) nnzL += (int64_t)(a - r) * (k - r);
        if (sf) {
          const int64_t m2 = r2 - r;
          nnzL += m2 * (k - r) - m2 * (m2 - 1) / 2;
        }
      }
    }

    if (apb) apb->publish(l);

    if (o.hbm_budget_bytes > 0) {
      // device memory held now: the factor so far, both row-panel buffers,
      // the scaling temporaries and the descriptor arenas
      const int64_t held = (int64_t)(F.arena.bytes_reserved() + F.meta.bytes_reserved() +
                                     C.panels[0].bytes + C.panels[1].bytes + C.temp.bytes);
      if (held > o.hbm_budget_bytes)
        throw Error(SPAND_E_OOM, "factorization needs more than hbm_budget_bytes (" +
                                     std::to_string(held) + " bytes held after step " +
                                     std::to_string(l) + ")");
    }

    if (stop_here) {
      F.stopped_at = l;
      F.dbg_layout = lay;
      F.dbg_ncur = cur_sizes;
      F.dbg_panels.resize(lay.total);
      std::vector<FT> dbg((size_t)lay.total);
      SPAND_HIP(hipMemcpy(dbg.data(), panel, lay.total * sizeof(FT), hipMemcpyDeviceToHost));
      std::copy(dbg.begin(), dbg.end(), F.dbg_panels.begin());
      break;
    }

    // no wait: the next step is planned while the merge runs (its uploads go
    // to the other descriptor arena)
    cur = 1 - cur;
    panel = npanel;
    lay_store = std::move(nlay);
    layp = &lay_store;
    sizes = std::move(nsz);
  }
  if (F.stopped_at < 0) {
    // triangular factors of the compact WY forms of every sparsified interface:
    // S = V^T V (lower triangle) by one batched GEMM, then the column recurrence
    // (more than kWyLdsN reflectors: the tiled inverse of T^-1, with an n x n
    // scratch each)
    C.upload.next(s);
    int64_t xdoubles = 0;
    for (const StepRec& R : F.steps)
      for (size_t p = 0; p < R.V.size(); ++p)
        if (R.V[p] && R.r2[p] > kWyLdsN) xdoubles += (int64_t)R.r2[p] * R.r2[p];
    FT* xs = xdoubles ? static_cast<FT*>(C.temp.ensure(xdoubles * sizeof(FT))) : nullptr;
    std::vector<GemmD> gd;
    std::vector<GemmTm> gt;
    std::vector<WyD> wy;
    for (const StepRec& R : F.steps) {
      for (size_t p = 0; p < R.V.size(); ++p) {
        if (!Pt(R.V[p]) || R.r2[p] <= 0) continue;
        const int nref = R.r2[p], a = R.n0[p];
        GemmD g{};
        g.C = Pt(R.T[p]);
        g.ldc = nref;
        g.m = nref;
        g.n = nref;
        g.transA = 1;
        g.transB = 0;
        g.lower_only = 1;
        g.alpha = 1.0;
        g.beta = 0.0;
        g.term0 = (int64_t)gt.size();
        gt.push_back(GemmTm{Pt(R.V[p]), Pt(R.V[p]), a, a, a, 0});
        g.term1 = (int64_t)gt.size();
        gd.push_back(g);
        FT* X = nullptr;
        if (nref > kWyLdsN) {
          X = xs;
          xs += (int64_t)nref * nref;
        }
        wy.push_back(WyD{Pt(R.V[p]), Pt(R.tau[p]), Pt(R.T[p]), X, a, nref});
      }
    }
    if (!wy.empty()) {
      run_gemm(C, o, gd, gt, s);
      const auto* d_wy = C.upload.upload(wy);
      SPAND_PROF(C, "k_wy_t", launch_wy_t(d_wy, (int32_t)wy.size(), s));
      // V T of every interface (a x nref): the apply then needs no pass over T
      // (Q^T x = x - V (VT)^T x, Q y = y - VT V^T y)
      std::vector<GemmD> gv;
      std::vector<GemmTm> gvt;
      for (const StepRec& R : F.steps)
        for (size_t p = 0; p < R.V.size(); ++p) {
          if (!Pt(R.V[p]) || R.r2[p] <= 0) continue;
          const int nref = R.r2[p], a = R.n0[p];
          GemmD g{};
          g.C = Pt(R.VT[p]);
          g.ldc = a;
          g.m = a;
          g.n = nref;
          g.alpha = 1.0;
          g.beta = 0.0;
          g.term0 = (int64_t)gvt.size();
          gvt.push_back(GemmTm{Pt(R.V[p]), Pt(R.T[p]), a, nref, nref, 0});
          g.term1 = (int64_t)gvt.size();
          gv.push_back(g);
        }
      run_gemm(C, o, gv, gvt, s);
    }
  }
  SPAND_HIP(hipStreamSynchronize(s));
  if (!deferred.empty()) throw Error(SPAND_E_STATE, "internal: breakdown flags left unchecked");
  if (apb && F.stopped_at < 0) {
    apb->finish();
    finish_apply(C, F);
  }
  F.stats.flops = flops;
  F.stats.nnz_L = nnzL;
  F.stats.factor_bytes = (int64_t)F.arena.bytes_used();
  F.stats.factor_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

void run_factor(Ctx& C, Plan& P, const double* d_vals, const spand_opts& o, FactorObj& F) {
  if (o.precision == SPAND_FP64) run_factor_t<double>(C, P, d_vals, o, F);
  else run_factor_t<float>(C, P, d_vals, o, F);
}

}  // namespace spand
