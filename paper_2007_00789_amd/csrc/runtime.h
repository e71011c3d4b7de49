// Context, device arenas and the numeric factor object (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace spand {

// Chunked bump allocator of device memory.  Chunks are kept until release();
// reset() makes every chunk reusable (the caller must have synchronized).
// A mirrored arena keeps a pinned host copy of every chunk: upload() writes
// the host side and marks it dirty, flush() issues one copy per dirty chunk.
class DevArena {
 public:
  explicit DevArena(bool mirrored = false) : mirrored_(mirrored) {}
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
  void flush(hipStream_t s);
  void reset() { cur_ = 0; used_ = 0; }
  void release();
  size_t bytes_reserved() const { return reserved_; }
  size_t bytes_used() const;

 private:
  struct Chunk { char* p; char* h; size_t size, lo, hi; };
  bool mirrored_;
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, used_ = 0, reserved_ = 0;
};

// A device buffer that only grows (contents are not preserved on growth).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
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

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  DevArena upload{true};   // per-step descriptors
  DevBuf panels[2];        // ping-pong row panels of consecutive steps
  DevBuf temp;             // scaling temporaries
  DevBuf ints;             // per-step integer outputs (n_cur, ranks, info)
  Prof prof;
};

// Host record of one step of a numeric factorization.  The apply replays the
// operations from these records (device pointers into the factor arena).
struct StepRec {
  int l = 0;
  bool sparsified = false;
  std::vector<int32_t> n0;                   // cluster sizes at step start
  std::vector<int32_t> r, r2, k;             // interfaces of sparsified steps (else -1)
  std::vector<int64_t> kmax;                 // interfaces: leading dimension of Y (W^T)
  std::vector<double*> Linv, G;              // interiors
  std::vector<int32_t> kint;                 // interiors: coupling width
  std::vector<double*> Zinv, Y, V, tau, T;   // interfaces of sparsified steps
  std::vector<double*> VT;                   // interfaces: V T (a x nref), for the apply
  std::vector<std::vector<int32_t>> pos;     // positions of each cluster's variables (step start)
  std::vector<std::vector<int32_t>> sp_nbr_pos;  // interfaces: positions of W's columns
};

struct FactorObj {
  Plan* plan = nullptr;
  spand_opts opts{};
  DevArena arena;                            // numeric factor data
  DevArena meta{true};                       // apply descriptors and position lists
  std::vector<StepRec> steps;                // indexed by l
  spand_factor_stats stats{};
  int stopped_at = -1;                       // debug stop step
  // debug: panel state of the stop step
  std::vector<double> dbg_panels;
  PanelLayout dbg_layout;
  std::vector<int32_t> dbg_ncur;
  // apply program (built by build_apply)
  struct ApplyProg* prog = nullptr;
  ~FactorObj();
};

// Thrown by run_factor when a cooperative QR group did not run on one XCD
// (its workgroups left without writing); the factorization is then redone with
// the single-workgroup QR.
struct CoopPlacement {};

void run_factor(Ctx& C, Plan& P, const double* d_vals, const spand_opts& o, FactorObj& F);

}  // namespace spand
