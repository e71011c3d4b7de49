// Serving loop (a project addition around the method): requests for solves
// with new or already factored matrices are admitted continuously by worker
// slots, each with its own context and stream.  A slot takes every admissible
// waiting request: the new matrices among them are analysed and factored
// together as one batch plan (spand_analyze_batch), their factors stay resident
// for later requests with the same key, and all the slot's requests on one
// factor are solved by one PCG call (one CG per problem and column; requests
// on different problems of a batch share columns).  Admission is by device
// footprint: new matrices are taken only if the estimate of their factors fits
// next to the resident ones within the byte budget, after the least recently
// used idle factors have been released.
//
// Overlap: the slots' analyses, uploads, factorizations and PCG solves run
// concurrently on their own streams; only the cooperative QR launches of the
// sparsified steps go one at a time per device (the library holds a device-wide
// lock from a step's first cooperative launch until its ranks are read back),
// because such a launch waits on workgroups of its own: two in flight could
// hold the compute units each other's groups need.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/spand.h"

namespace {

using Clock = std::chrono::steady_clock;

// host copy of a matrix, kept so that its factor can be rebuilt after release
struct Matrix {
  int64_t n = 0;
  int32_t dim = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<double> coords, vals;
  int64_t est_bytes = 0;
};

struct Request {
  int64_t id = 0, key = 0;
  int32_t nrhs = 0;
  std::vector<double> b, x, relres;
  std::vector<int32_t> iters;
  Clock::time_point t_submit;
  double latency = 0.0;
  spand_status status = SPAND_OK;
  bool done = false;
};

// the factor of one batch of matrices, resident on the device
struct Resident {
  spand_plan_t plan = nullptr;
  spand_factor_t fac = nullptr;
  std::vector<int64_t> seg_off, keys;
  int64_t bytes = 0;
  bool busy = false;   // claimed by a slot (guarded by the server mutex)
  Clock::time_point last_use;
  ~Resident() {
    if (fac) spand_destroy_factor(fac);
    if (plan) spand_destroy_plan(plan);
  }
};

// device bytes of a factor are estimated from nnz(A) before it exists: the
// sparsified factor of a 3D problem holds about 80 entries per nonzero of A
constexpr int64_t kEstEntriesPerNnz = 96;

}  // namespace

struct spand_server_s {
  int device = 0;
  spand_opts opts{};
  double tol = 1e-10;
  int32_t maxit = 1000;
  int64_t max_bytes = 0;
  int32_t max_batch = 32;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  int64_t next_id = 1;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> requests;
  std::unordered_map<int64_t, Matrix> matrices;
  std::unordered_map<int64_t, std::pair<std::shared_ptr<Resident>, int>> where;  // key -> factor, problem
  std::unordered_map<int64_t, int> in_flight;                                    // keys being factored
  std::vector<std::shared_ptr<Resident>> residents;
  int64_t resident_bytes = 0, reserved_bytes = 0;
  int64_t factor_batches = 0, factored_matrices = 0, pcg_calls = 0;
  double analyze_s = 0.0, factor_s = 0.0, pcg_s = 0.0;   // summed over slots
  std::vector<std::thread> workers;
  std::vector<spand_ctx_t> ctxs;
  std::vector<hipStream_t> streams;
  std::string error;

  void worker(spand_ctx_t ctx, hipStream_t stream);
  void release_idle(int64_t need);
  void take_batch(std::vector<std::shared_ptr<Request>>& out, std::vector<int64_t>& new_keys,
                  std::vector<std::shared_ptr<Resident>>& claimed, int64_t& reserved);
};

void spand_server_s::release_idle(int64_t need) {
  while (resident_bytes + reserved_bytes + need > max_bytes) {
    auto it = std::min_element(residents.begin(), residents.end(), [](const auto& a, const auto& b) {
      if (a->busy != b->busy) return !a->busy;
      return a->last_use < b->last_use;
    });
    if (it == residents.end() || (*it)->busy) return;
    for (int64_t k : (*it)->keys) where.erase(k);
    resident_bytes -= (*it)->bytes;
    residents.erase(it);   // destroyed here unless a slot still holds it
  }
}

// Takes the admissible waiting requests, oldest first (server mutex held):
// requests on a resident factor no other slot is using, and requests with new
// matrices whose estimated footprint fits the budget.
void spand_server_s::take_batch(std::vector<std::shared_ptr<Request>>& out,
                                std::vector<int64_t>& new_keys,
                                std::vector<std::shared_ptr<Resident>>& claimed, int64_t& reserved) {
  reserved = 0;
  for (auto it = queue.begin(); it != queue.end() && (int)out.size() < max_batch;) {
    const auto& r = *it;
    bool take = false;
    auto w = where.find(r->key);
    if (w != where.end()) {
      const auto& f = w->second.first;
      const bool mine = std::find(claimed.begin(), claimed.end(), f) != claimed.end();
      if (mine || !f->busy) {
        if (!mine) {
          f->busy = true;
          claimed.push_back(f);
        }
        take = true;
      }
    } else if (std::find(new_keys.begin(), new_keys.end(), r->key) != new_keys.end()) {
      take = true;   // its matrix is already in this batch
    } else if (!in_flight.count(r->key)) {
      const int64_t e = matrices[r->key].est_bytes;
      release_idle(reserved + e);
      const bool alone = out.empty() && residents.empty() && reserved_bytes == 0;
      if (resident_bytes + reserved_bytes + reserved + e <= max_bytes || alone) {
        new_keys.push_back(r->key);
        reserved += e;
        take = true;
      }
    }
    if (take) {
      out.push_back(r);
      it = queue.erase(it);
    } else {
      ++it;
    }
  }
  for (int64_t k : new_keys) in_flight[k] = 1;
  reserved_bytes += reserved;
}

void spand_server_s::worker(spand_ctx_t ctx, hipStream_t stream) {
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    std::vector<int64_t> new_keys;
    std::vector<std::shared_ptr<Resident>> claimed;
    int64_t reserved = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) break;
      take_batch(batch, new_keys, claimed, reserved);
      if (batch.empty()) {
        // everything waiting needs a factor another slot holds or memory
        // another slot will release: wait for a slot to finish
        cv_done.wait_for(lk, std::chrono::milliseconds(5));
        continue;
      }
    }
    std::string msg;
    // the new matrices: one batch plan, one factorization
    spand_status fst = SPAND_OK;
    if (!new_keys.empty()) {
      auto fresh = std::make_shared<Resident>();
      std::vector<const Matrix*> ms;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (int64_t k : new_keys) ms.push_back(&matrices.at(k));   // nodes are stable
      }
      const int cnt = (int)ms.size();
      std::vector<int64_t> ns(cnt);
      std::vector<const int64_t*> rp(cnt);
      std::vector<const int32_t*> ci(cnt);
      std::vector<const double*> xy(cnt);
      std::vector<int32_t> dims(cnt);
      int64_t nnz = 0, n = 0;
      for (int i = 0; i < cnt; ++i) {
        ns[i] = ms[i]->n;
        rp[i] = ms[i]->rowptr.data();
        ci[i] = ms[i]->colind.data();
        xy[i] = ms[i]->coords.data();
        dims[i] = ms[i]->dim;
        nnz += (int64_t)ms[i]->colind.size();
        n += ms[i]->n;
      }
      const auto ta = Clock::now();
      fst = spand_analyze_batch(ctx, cnt, ns.data(), rp.data(), ci.data(), xy.data(), dims.data(),
                                nullptr, &opts, &fresh->plan);
      const auto tb = Clock::now();
      double* d_vals = nullptr;
      if (fst == SPAND_OK && hipMalloc(&d_vals, std::max<int64_t>(nnz, 1) * sizeof(double)) != hipSuccess)
        fst = SPAND_E_OOM;
      for (int i = 0, o = 0; fst == SPAND_OK && i < cnt; o += (int)ms[i]->vals.size(), ++i)
        if (hipMemcpyAsync(d_vals + o, ms[i]->vals.data(), ms[i]->vals.size() * sizeof(double),
                           hipMemcpyHostToDevice, stream) != hipSuccess)
          fst = SPAND_E_HIP;
      double tf = 0.0;
      if (fst == SPAND_OK) {
        const auto t1 = Clock::now();
        fst = spand_factor(ctx, fresh->plan, d_vals, &opts, &fresh->fac);
        tf = std::chrono::duration<double>(Clock::now() - t1).count();
      }
      if (d_vals) (void)hipFree(d_vals);   // the factor holds its own copy of the values
      if (fst == SPAND_OK) {
        int32_t nseg = 0;
        spand_plan_segments(fresh->plan, &nseg, nullptr);
        fresh->seg_off.resize(nseg + 1);
        spand_plan_segments(fresh->plan, &nseg, fresh->seg_off.data());
        spand_factor_stats fs{};
        spand_factor_info(fresh->fac, &fs);
        // factor, its values and the plan's device arrays
        fresh->bytes = fs.factor_bytes + nnz * 28 + n * 12;
        fresh->keys = new_keys;
        fresh->busy = true;
      } else {
        msg = spand_last_error(ctx);
      }
      std::lock_guard<std::mutex> lk(mu);
      analyze_s += std::chrono::duration<double>(tb - ta).count();
      factor_s += tf;
      reserved_bytes -= reserved;
      for (int64_t k : new_keys) in_flight.erase(k);
      if (fst == SPAND_OK) {
        resident_bytes += fresh->bytes;
        residents.push_back(fresh);
        claimed.push_back(fresh);
        for (int i = 0; i < cnt; ++i) where[new_keys[i]] = {fresh, i};
        ++factor_batches;
        factored_matrices += cnt;
      }
    }
    // group the requests by factor; columns: the requests on one problem
    // take consecutive columns, requests on different problems share them
    struct Slot {
      std::shared_ptr<Request> r;
      int seg, col;
    };
    std::map<Resident*, std::vector<Slot>> groups;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto& r : batch) {
        auto w = where.find(r->key);
        if (w == where.end()) {   // its factorization failed in this batch
          r->status = fst != SPAND_OK ? fst : SPAND_E_STATE;
          continue;
        }
        groups[w->second.first.get()].push_back({r, w->second.second, 0});
      }
    }
    for (auto& [f, slots] : groups) {
      const int64_t n = f->seg_off.back();
      const int nseg = (int)f->seg_off.size() - 1;
      std::vector<int32_t> used(nseg, 0);
      int32_t cols = 0;
      for (auto& s : slots) {
        s.col = used[s.seg];
        used[s.seg] += s.r->nrhs;
        cols = std::max(cols, used[s.seg]);
      }
      std::vector<double> hb((size_t)n * cols, 0.0);
      for (auto& s : slots) {
        const int64_t o = f->seg_off[s.seg], len = f->seg_off[s.seg + 1] - o;
        for (int c = 0; c < s.r->nrhs; ++c)
          std::memcpy(&hb[(size_t)(s.col + c) * n + o], &s.r->b[(size_t)c * len], len * sizeof(double));
      }
      double *db = nullptr, *dx = nullptr;
      spand_status ps = SPAND_OK;
      if (hipMalloc(&db, hb.size() * sizeof(double)) != hipSuccess ||
          hipMalloc(&dx, hb.size() * sizeof(double)) != hipSuccess)
        ps = SPAND_E_OOM;
      if (ps == SPAND_OK && hipMemcpyAsync(db, hb.data(), hb.size() * sizeof(double),
                                           hipMemcpyHostToDevice, stream) != hipSuccess)
        ps = SPAND_E_HIP;
      std::vector<int32_t> it((size_t)nseg * cols, 0);
      std::vector<double> rr((size_t)nseg * cols, 0.0);
      const auto tp = Clock::now();
      if (ps == SPAND_OK) {
        ps = spand_pcg(ctx, f->fac, cols, db, dx, tol, maxit, it.data(), rr.data());
        if (ps != SPAND_OK && ps != SPAND_E_NO_CONVERGENCE) msg = spand_last_error(ctx);
      }
      if ((ps == SPAND_OK || ps == SPAND_E_NO_CONVERGENCE) &&
          (hipMemcpyAsync(hb.data(), dx, hb.size() * sizeof(double), hipMemcpyDeviceToHost, stream) !=
               hipSuccess ||
           hipStreamSynchronize(stream) != hipSuccess))
        ps = SPAND_E_HIP;
      if (db) (void)hipFree(db);
      if (dx) (void)hipFree(dx);
      std::lock_guard<std::mutex> lk(mu);
      ++pcg_calls;
      pcg_s += std::chrono::duration<double>(Clock::now() - tp).count();
      for (auto& s : slots) {
        Request& r = *s.r;
        const int64_t o = f->seg_off[s.seg], len = f->seg_off[s.seg + 1] - o;
        r.status = ps == SPAND_E_NO_CONVERGENCE ? SPAND_OK : ps;
        if (r.status != SPAND_OK) continue;
        r.x.resize((size_t)len * r.nrhs);
        r.iters.resize(r.nrhs);
        r.relres.resize(r.nrhs);
        for (int c = 0; c < r.nrhs; ++c) {
          std::memcpy(&r.x[(size_t)c * len], &hb[(size_t)(s.col + c) * n + o], len * sizeof(double));
          r.iters[c] = it[(size_t)s.seg * cols + s.col + c];
          r.relres[c] = rr[(size_t)s.seg * cols + s.col + c];
          if (r.iters[c] >= maxit) r.status = SPAND_E_NO_CONVERGENCE;
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      const auto now = Clock::now();
      for (auto& f : claimed) {
        f->busy = false;
        f->last_use = now;
      }
      for (auto& r : batch) {
        r->latency = std::chrono::duration<double>(now - r->t_submit).count();
        r->done = true;
      }
      if (!msg.empty()) error = msg;
    }
    cv_done.notify_all();
    cv.notify_all();
  }
}

extern "C" {

spand_status spand_server_create(int32_t device, const spand_opts* opts, double tol, int32_t maxit,
                                 int64_t max_bytes, int32_t slots, int32_t max_batch,
                                 spand_server_t* out) {
  if (!out) return SPAND_E_INVALID;
  *out = nullptr;
  if (!opts || slots < 1 || slots > 16 || max_batch < 1 || max_bytes <= 0 || !(tol > 0.0) ||
      maxit < 1)
    return SPAND_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return SPAND_E_HIP;
  if (device < 0 || device >= ndev) return SPAND_E_INVALID;
  auto* s = new spand_server_s();
  s->device = device;
  s->opts = *opts;
  s->tol = tol;
  s->maxit = maxit;
  s->max_bytes = max_bytes;
  s->max_batch = max_batch;
  // one context and stream per slot
  spand_status st = SPAND_OK;
  for (int i = 0; i < slots && st == SPAND_OK; ++i) {
    hipStream_t stream = nullptr;
    spand_ctx_t ctx = nullptr;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
      st = SPAND_E_HIP;
    } else if ((st = spand_create(&ctx, device, stream)) != SPAND_OK) {
      (void)hipStreamDestroy(stream);
    } else {
      s->streams.push_back(stream);
      s->ctxs.push_back(ctx);
    }
  }
  if (st != SPAND_OK) {
    for (auto c : s->ctxs) spand_destroy(c);
    for (auto q : s->streams) (void)hipStreamDestroy(q);
    delete s;
    return st;
  }
  for (int i = 0; i < slots; ++i)
    s->workers.emplace_back([s, i] { s->worker(s->ctxs[i], s->streams[i]); });
  *out = s;
  return SPAND_OK;
}

spand_status spand_server_submit(spand_server_t s, int64_t key, int64_t n, const int64_t* rowptr,
                                 const int32_t* colind, const double* coords, int32_t dim,
                                 const double* vals, int32_t nrhs, const double* b,
                                 int64_t* req_id) {
  if (!s || !b || nrhs < 1 || !req_id) return SPAND_E_INVALID;
  auto r = std::make_shared<Request>();
  r->key = key;
  r->nrhs = nrhs;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) return SPAND_E_STATE;
  auto m = s->matrices.find(key);
  if (m == s->matrices.end()) {
    // a new key brings its matrix; it is copied here and checked by the analysis
    if (n <= 0 || !rowptr || !colind || !coords || !vals || dim < 1 || dim > 3 || rowptr[0] != 0 ||
        rowptr[n] < n)
      return SPAND_E_INVALID;
    Matrix mt;
    mt.n = n;
    mt.dim = dim;
    mt.rowptr.assign(rowptr, rowptr + n + 1);
    mt.colind.assign(colind, colind + rowptr[n]);
    mt.coords.assign(coords, coords + n * dim);
    mt.vals.assign(vals, vals + rowptr[n]);
    mt.est_bytes = rowptr[n] * kEstEntriesPerNnz * (int64_t)sizeof(double);
    m = s->matrices.emplace(key, std::move(mt)).first;
  } else if (n > 0 && n != m->second.n) {
    return SPAND_E_INVALID;
  }
  r->b.assign(b, b + (size_t)m->second.n * nrhs);
  r->id = s->next_id++;
  r->t_submit = Clock::now();
  s->requests[r->id] = r;
  s->queue.push_back(r);
  *req_id = r->id;
  lk.unlock();
  s->cv.notify_one();
  return SPAND_OK;
}

spand_status spand_server_poll(spand_server_t s, int64_t req_id, int32_t wait, int32_t* done,
                               double* x, int32_t* iters, double* relres, double* latency) {
  if (!s || !done) return SPAND_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(req_id);
  if (it == s->requests.end()) return SPAND_E_INVALID;
  auto r = it->second;
  if (wait) s->cv_done.wait(lk, [&] { return r->done; });
  *done = r->done ? 1 : 0;
  if (!r->done) return SPAND_OK;
  if (!r->x.empty()) {
    if (x) std::memcpy(x, r->x.data(), r->x.size() * sizeof(double));
    if (iters) std::memcpy(iters, r->iters.data(), r->nrhs * sizeof(int32_t));
    if (relres) std::memcpy(relres, r->relres.data(), r->nrhs * sizeof(double));
  }
  if (latency) *latency = r->latency;
  const spand_status st = r->status;
  s->requests.erase(it);
  return st;
}

spand_status spand_server_stats(spand_server_t s, int64_t* counters) {
  if (!s || !counters) return SPAND_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  counters[0] = s->resident_bytes;
  counters[1] = (int64_t)s->residents.size();
  counters[2] = (int64_t)s->queue.size();
  counters[3] = s->factor_batches;
  counters[4] = s->factored_matrices;
  counters[5] = s->pcg_calls;
  counters[6] = (int64_t)(s->analyze_s * 1e6);
  counters[7] = (int64_t)(s->factor_s * 1e6);
  counters[8] = (int64_t)(s->pcg_s * 1e6);
  return SPAND_OK;
}

const char* spand_server_error(spand_server_t s) { return s ? s->error.c_str() : ""; }

void spand_server_destroy(spand_server_t s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  s->where.clear();
  s->residents.clear();
  for (auto c : s->ctxs) spand_destroy(c);
  for (auto q : s->streams) (void)hipStreamDestroy(q);
  delete s;
}

}  // extern "C"
