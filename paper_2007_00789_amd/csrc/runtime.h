// Context, device arenas and the numeric factor object (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace spand {

// Pinned host staging memory for asynchronous uploads.  Everything staged
// stays valid until reset(), which the caller issues only after the stream
// has synchronized.
class PinnedArena {
 public:
  PinnedArena() = default;
  PinnedArena(const PinnedArena&) = delete;
  PinnedArena& operator=(const PinnedArena&) = delete;
  ~PinnedArena() { release(); }
  void* alloc(size_t bytes);
  void reset() { cur_ = 0; used_ = 0; }
  void release();

 private:
  struct Chunk { char* p; size_t size; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, used_ = 0;
};

// Chunked bump allocator of device memory.  Chunks are kept until release();
// reset() makes every chunk reusable (the caller must have synchronized).
class DevArena {
 public:
  DevArena() = default;
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  ~DevArena() { release(); }
  void* alloc(size_t bytes);
  template <class T>
  T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  // copies v through pinned staging memory (valid until stage.reset())
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s, PinnedArena& stage) {
    if (v.empty()) return nullptr;
    T* d = alloc_n<T>(v.size());
    void* h = stage.alloc(v.size() * sizeof(T));
    std::memcpy(h, v.data(), v.size() * sizeof(T));
    SPAND_HIP(hipMemcpyAsync(d, h, v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
  }
  void reset() { cur_ = 0; used_ = 0; }
  void release();
  size_t bytes_reserved() const { return reserved_; }
  size_t bytes_used() const;

 private:
  struct Chunk { char* p; size_t size; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, used_ = 0, reserved_ = 0;
  size_t used_before_ = 0;
};

// A device buffer that only grows (contents are not preserved on growth).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* ensure(size_t need);
  void release();
  ~DevBuf() { release(); }
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  DevArena upload;         // per-step descriptors
  PinnedArena stage;       // host side of every upload
  DevBuf panels[2];        // ping-pong row panels of consecutive steps
  DevBuf temp;             // scaling temporaries
  DevBuf ints;             // per-step integer outputs (n_cur, ranks, info)
};

// Host record of one step of a numeric factorization.  The apply replays the
// operations from these records (device pointers into the factor arena).
struct StepRec {
  int l = 0;
  bool sparsified = false;
  std::vector<int32_t> n0;                   // cluster sizes at step start
  std::vector<int32_t> r, r2, k;             // interfaces of sparsified steps (else -1)
  std::vector<double*> Linv, G;              // interiors
  std::vector<int32_t> kint;                 // interiors: coupling width
  std::vector<double*> Zinv, Y, V, tau;      // interfaces of sparsified steps
  std::vector<std::vector<int32_t>> pos;     // positions of each cluster's variables (step start)
  std::vector<std::vector<int32_t>> sp_nbr_pos;  // interfaces: positions of W's columns
};

struct FactorObj {
  Plan* plan = nullptr;
  spand_opts opts{};
  DevArena arena;
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

void run_factor(Ctx& C, Plan& P, const double* d_vals, const spand_opts& o, FactorObj& F);

}  // namespace spand
