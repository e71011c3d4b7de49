// Context, device arenas and the numeric factor object (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace spand {

// Device chunks (with their pinned host mirrors, for mirrored arenas) kept
// for reuse by the arenas of later factorizations and solves on one device, so
// that a factor-solve cycle does not pay hipMalloc / hipFree (which waits for
// the device) for its large buffers.  Holds at most `cap` idle bytes; beyond
// that, returned chunks are freed.  Thread-safe (factors may be destroyed on
// any thread); owned jointly by the context and the arenas drawing from it.
class MemPool {
 public:
  MemPool(int device, size_t cap) : device_(device), cap_(cap) {}
  MemPool(const MemPool&) = delete;
  MemPool& operator=(const MemPool&) = delete;
  ~MemPool();
  // a chunk of at least `bytes` (the smallest idle one), or false
  bool take(size_t bytes, bool mirrored, char** dev, char** host, size_t* size);
  void give(char* dev, char* host, size_t size);

 private:
  struct Chunk { char* d; char* h; size_t size; };
  std::mutex mu_;
  std::vector<Chunk> idle_;
  int device_;
  size_t cap_, held_ = 0;
};

// Chunked bump allocator of device memory.  Chunks are kept until release();
// reset() makes every chunk reusable (the caller must have synchronized).
// A mirrored arena keeps a pinned host copy of every chunk: upload() writes
// the host side and marks it dirty, flush() issues one copy per dirty chunk.
class DevArena {
 public:
  explicit DevArena(bool mirrored = false) : mirrored_(mirrored) {}
  // chunks come from and go back to `pool` (nullptr: hipMalloc / hipFree)
  void set_pool(std::shared_ptr<MemPool> pool) { pool_ = std::move(pool); }
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  ~DevArena() { release(); }
  void* alloc(size_t bytes);
  template <class T>
  T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  // device address of a copy of v (valid on the device after flush())
  template <class T>
  T* upload(const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    T* d = alloc_n<T>(v.size());
    Chunk& c = chunks_[cur_];
    const size_t off = reinterpret_cast<char*>(d) - c.p, bytes = v.size() * sizeof(T);
    std::memcpy(c.h + off, v.data(), bytes);
    c.lo = std::min(c.lo, off);
    c.hi = std::max(c.hi, off + bytes);
    return d;
  }
  // room for n elements to be written in place in the pinned host copy:
  // returns their host address and sets *dev to the device address;
  // commit(h, count) then includes the first count of them in the next flush
  template <class T>
  T* stage(size_t n, T** dev) {
    T* d = alloc_n<T>(std::max<size_t>(n, 1));
    const Chunk& c = chunks_[cur_];
    *dev = d;
    return reinterpret_cast<T*>(c.h + (reinterpret_cast<char*>(d) - c.p));
  }
  template <class T>
  void commit(const T* h, size_t count) { mark(reinterpret_cast<const char*>(h), count * sizeof(T)); }
  void flush(hipStream_t s);
  void reset() { cur_ = 0; used_ = 0; }
  void release();
  size_t bytes_reserved() const { return reserved_; }
  size_t bytes_used() const;

 private:
  struct Chunk { char* p; char* h; size_t size, lo, hi; };
  void mark(const char* h, size_t bytes);
  bool mirrored_;
  std::shared_ptr<MemPool> pool_;
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, used_ = 0, reserved_ = 0;
};

// Two mirrored descriptor arenas used by alternate steps of the factorization:
// a step's uploads may still be in flight on the stream while the host plans
// the next step.  Switching arenas records an event on the stream for the one
// left; an arena is reset only after the event of its previous use has
// completed (the host waits there when the device is more than a step behind).
class UploadRing {
 public:
  UploadRing() = default;
  UploadRing(const UploadRing&) = delete;
  UploadRing& operator=(const UploadRing&) = delete;
  ~UploadRing();
  template <class T>
  T* upload(const std::vector<T>& v) { return a_[cur_].upload(v); }
  // device-only scratch of the current step (never in an uploaded range, so
  // no flush overwrites it)
  template <class T>
  T* scratch_n(size_t n) { return s_[cur_].alloc_n<T>(n); }
  template <class T>
  T* stage(size_t n, T** dev) { return a_[cur_].stage<T>(n, dev); }
  template <class T>
  void commit(const T* h, size_t count) { a_[cur_].commit(h, count); }
  void flush(hipStream_t s) { a_[cur_].flush(s); }
  // switch to the other arena and make all of it reusable once the copies
  // and kernels that read it before have completed
  void next(hipStream_t s);

 private:
  DevArena a_[2] = {DevArena(true), DevArena(true)};
  DevArena s_[2];
  hipEvent_t ev_[2] = {nullptr, nullptr};
  bool used_[2] = {false, false};
  int cur_ = 0;
};

// A device buffer that only grows (contents are not preserved on growth).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::shared_ptr<MemPool> pool;   // nullptr: hipMalloc / hipFree
  void* ensure(size_t need);
  void release();
  ~DevBuf() { release(); }
};

// Opt-in per-kernel timing: HIP events recorded on the launch stream around
// every launch, resolved after the enclosing call has synchronized.
struct Prof {
  struct Entry { std::string name; double ms = 0.0; int64_t calls = 0; double work = 0.0; };
  bool on = false;
  std::string only;   // non-empty: time this kernel name only
  std::vector<Entry> entries;
  struct Pending { int entry; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int find(const char* name);
  int begin(const char* name, hipStream_t s);
  void end(int id, hipStream_t s);
  void add_work(const char* name, double w);
  // the work of `name` is recorded (callers skip computing it otherwise)
  bool wants(const char* name) const { return on && (only.empty() || only == name); }
  void resolve();   // caller has synchronized the stream
  void reset();
  ~Prof();
};

// Flushes the pending descriptor uploads, then times the launch.  The
// statement itself must not upload: every descriptor it reads has to be
// uploaded before the macro so that the flush covers it.
#define SPAND_PROF(C, name, stmt)                      \
  do {                                                 \
    (C).upload.flush((C).stream);                      \
    const int pid_ = (C).prof.begin(name, (C).stream); \
    stmt;                                              \
    (C).prof.end(pid_, (C).stream);                    \
  } while (0)

// Tile choice of the batched GEMM per size class of the launch's output blocks
// and per element type (index 0: double, 1: float), measured on the device.
struct GemmTuner {
  static constexpr int kClasses = 4;
  bool tuned[2] = {false, false};
  int tile[2][kClasses] = {{64, 64, 64, 64}, {64, 64, 64, 64}};
  float ms[2][kClasses][2] = {};   // trial times, 64- and 128-tile kernels
};

// Size of the fixed device scratch of the allocation-free apply (one array per
// device, held until the process ends).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;

struct Ctx {
  int device = 0;
  void* noalloc = nullptr; // device address of the fixed apply scratch of this device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  std::shared_ptr<MemPool> pool;   // chunks of factor and solve arenas
  UploadRing upload;       // per-step descriptors (two arenas, alternate steps)
  DevBuf panels[2];        // ping-pong row panels of consecutive steps
  DevBuf temp;             // scaling temporaries
  DevBuf ints;             // per-step integer outputs (n_cur, ranks, info)
  GemmTuner tuner;         // GEMM tile per size class (measured at the first factorization)
  Prof prof;
};

// Variables of every cluster of one step, flat: cluster c holds
// idx[ptr[c] .. ptr[c+1]).
struct PosLists {
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  const int32_t* begin(int c) const { return idx.data() + ptr[c]; }
  int32_t size(int c) const { return (int32_t)(ptr[c + 1] - ptr[c]); }
};

// Host record of one step of a numeric factorization.  The apply replays the
// operations from these records (device pointers into the factor arena).
struct StepRec {
  int l = 0;
  bool sparsified = false;
  std::vector<int32_t> n0;                   // cluster sizes at step start
  std::vector<int32_t> r, r2, k;             // interfaces of sparsified steps (else -1)
  std::vector<int64_t> kmax;                 // interfaces: leading dimension of Y (W^T)
  // factor entries: double, or float when FactorObj::f32
  std::vector<void*> Linv, G;                // interiors
  std::vector<int32_t> kint;                 // interiors: coupling width
  std::vector<void*> Zinv, Y, V, tau, T;     // interfaces of sparsified steps
  std::vector<void*> VT;                     // interfaces: V T (a x nref), for the apply
  PosLists pos;                              // positions of each cluster's variables (step start)
  PosLists sp_nbr_pos;                       // interfaces: positions of W's columns
};

struct FactorObj {
  Plan* plan = nullptr;
  bool f32 = false;                          // factor entries are float (FP32 precisions)
  spand_opts opts{};
  std::shared_ptr<MemPool> arena_pool;       // the context's pool (chunks of the buffers below)
  DevArena arena;                            // numeric factor data
  DevArena meta{true};                       // apply descriptors and position lists
  std::vector<StepRec> steps;                // indexed by l
  spand_factor_stats stats{};
  int stopped_at = -1;                       // debug stop step
  // debug: panel state of the stop step
  std::vector<double> dbg_panels;
  PanelLayout dbg_layout;
  std::vector<int32_t> dbg_ncur;
  // apply program (built step by step during run_factor)
  struct ApplyProg* prog = nullptr;
  // prescale: D^{-1/2} (n, device; owned by the caller of run_factor), or nullptr
  const double* dscale = nullptr;
  ~FactorObj();
};

// Thrown by run_factor when a cooperative QR group did not run on one XCD
// (its workgroups left without writing); the factorization is then redone with
// the single-workgroup QR.
struct CoopPlacement {};

// Factorization (Alg. 2); builds the apply program too unless stopped early.
void run_factor(Ctx& C, Plan& P, const double* d_vals, const spand_opts& o, FactorObj& F);
// apply program: a fresh one, the records of step l (steps in order D ... 0),
// then the upload of its descriptors
void begin_apply(FactorObj& F);
void build_apply_step(FactorObj& F, int l);
void finish_apply(Ctx& C, FactorObj& F);
// device address of the fixed scratch array on `device` (current), looked up
// once per device
void* noalloc_scratch(int device);
// y = M x with every temporary in the fixed scratch (no device allocation);
// SPAND_E_LIMIT when one column needs more than kNoAllocScratchBytes
void run_apply_noalloc(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y);

}  // namespace spand
