// C ABI of libspand: argument checking, error translation and object lifetime.
#include <algorithm>
#include <atomic>
#include <exception>
#include <thread>
#include <vector>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "apply.h"
#include "runtime.h"

// idle device memory a context keeps for the next factorization or solve
constexpr size_t kPoolIdleBytes = size_t(16) << 30;
struct spand_plan_s {
  spand::Plan p;
  uint64_t id = 0;   // unique per plan object (keys the context's merged-plan cache)
};
// A numeric factor: one problem's, or one batch's (the problems of a
// spand_factor_batch call), with the plan it was computed on.
struct FactorCore {
  spand::FactorObj f;
  spand::DevBuf vals;        // copy of A's values (SpMV inside PCG)
  double* d_vals = nullptr;  // = vals.p
  spand::DevBuf dscale;      // prescale: D^{-1/2} (n)
  int device = 0;
  std::shared_ptr<spand::Plan> merged;   // batch factors: the merged plan (f.plan points to it)
};
// A factor handle: the whole core (seg < 0), or problem seg of a batch core.
struct spand_factor_s {
  std::shared_ptr<FactorCore> core;
  int seg = -1;
  // seg >= 0: the problem's own rows, depth and clusters per own step
  int64_t n = 0, row0 = 0;
  int depth = 0;
  std::vector<int32_t> nI, nc;
  spand::FactorObj& F() { return core->f; }
};
struct spand_ctx_s {
  spand::Ctx c;
  // merged plan of the last spand_factor_batch call and the plan ids it was built from
  std::vector<uint64_t> batch_key;
  std::shared_ptr<spand::Plan> batch_plan;
  spand::DevBuf vtmp[2];    // handles of a batch factor: problem vectors embedded in batch vectors
};

namespace spand {
void run_apply(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y);
void run_pcg(Ctx& C, FactorObj& F, const double* d_vals, int32_t nrhs, const double* b, double* x,
             double tol, int32_t maxit, int32_t* iters, double* relres, bool* converged);
}  // namespace spand

namespace {

std::atomic<uint64_t> g_plan_ids{1};

template <class F>
spand_status guarded(spand_ctx_t ctx, F&& fn) {
  try {
    fn();
    if (ctx) ctx->c.last_error.clear();
    return SPAND_OK;
  } catch (const spand::Error& e) {
    if (ctx) ctx->c.last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.last_error = "host allocation failed";
    return SPAND_E_OOM;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.last_error = e.what();
    return SPAND_E_STATE;
  }
}

void check_opts(const spand_opts* o) {
  using spand::Error;
  if (!o) throw Error(SPAND_E_INVALID, "opts is NULL");
  if (!(o->eps >= 0.0 && o->eps <= 1.0)) throw Error(SPAND_E_INVALID, "eps must lie in [0, 1]");
  if (o->scheme < SPAND_FIRST_ORDER || o->scheme > SPAND_SUPERFINE)
    throw Error(SPAND_E_INVALID, "unknown scheme");
  if (o->skip < 0) throw Error(SPAND_E_INVALID, "skip must be >= 0");
  if (o->precision != SPAND_FP64 && o->precision != SPAND_FP32 && o->precision != SPAND_FP32_BF16)
    throw Error(SPAND_E_INVALID, "unknown precision");
  if (o->qr_group < -1 || o->qr_list_cap < -1 || o->qr_list_cap > 32 || o->qr_xcd_local < 0 ||
      o->qr_xcd_local > 1 || o->qr_lds_cols < 0 || o->qr_single_launch < 0 ||
      o->qr_single_launch > 1)
    throw Error(SPAND_E_INVALID, "bad QR testing options");
  if (o->prescale < 0 || o->prescale > 1) throw Error(SPAND_E_INVALID, "prescale must be 0 or 1");
  if (o->top_fp64_levels < 0) throw Error(SPAND_E_INVALID, "top_fp64_levels must be >= 0");
  if (o->hbm_budget_bytes < 0) throw Error(SPAND_E_INVALID, "hbm_budget_bytes must be >= 0");
  if (o->apply_graph < 0 || o->apply_graph > 1) throw Error(SPAND_E_INVALID, "apply_graph must be 0 or 1");
  if (o->gemm_tile != 0 && o->gemm_tile != 64 && o->gemm_tile != 128)
    throw Error(SPAND_E_INVALID, "gemm_tile must be 0, 64 or 128");
}

// device copies of the pattern and of the leaf assembly map, made on first use
void upload_plan(spand::Plan& P, int device) {
  if (P.d_rowptr) {
    if (P.device != device) throw spand::Error(SPAND_E_STATE, "plan is bound to another device");
    return;
  }
  P.device = device;
  SPAND_HIP(hipMalloc(&P.d_rowptr, (P.n + 1) * sizeof(int64_t)));
  SPAND_HIP(hipMalloc(&P.d_colind, std::max<int64_t>(P.nnz, 1) * sizeof(int32_t)));
  SPAND_HIP(hipMalloc(&P.d_leaf_dest, std::max<int64_t>(P.nnz, 1) * sizeof(int64_t)));
  SPAND_HIP(hipMemcpy(P.d_rowptr, P.rowptr.data(), (P.n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  SPAND_HIP(hipMemcpy(P.d_colind, P.colind.data(), P.nnz * sizeof(int32_t), hipMemcpyHostToDevice));
  SPAND_HIP(hipMemcpy(P.d_leaf_dest, P.leaf_dest.data(), P.nnz * sizeof(int64_t),
                      hipMemcpyHostToDevice));
  SPAND_HIP(hipMalloc(&P.d_seg_off, P.seg_off.size() * sizeof(int64_t)));
  SPAND_HIP(hipMemcpy(P.d_seg_off, P.seg_off.data(), P.seg_off.size() * sizeof(int64_t),
                      hipMemcpyHostToDevice));
  if (!P.seg_id.empty()) {
    SPAND_HIP(hipMalloc(&P.d_seg_id, P.n * sizeof(int32_t)));
    SPAND_HIP(hipMemcpy(P.d_seg_id, P.seg_id.data(), P.n * sizeof(int32_t), hipMemcpyHostToDevice));
  }
}

}  // namespace

extern "C" {

void spand_default_opts(spand_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->depth = 0;
  o->skip = 4;
  o->eps = 1e-2;
  o->scheme = SPAND_SECOND_ORDER;
  o->precision = SPAND_FP64;
  o->debug_stop_step = -1;
  o->qr_group = 0;
  o->qr_list_cap = -1;
  o->qr_xcd_local = 1;
  o->qr_lds_cols = 0;
  o->prescale = 0;
  o->top_fp64_levels = 3;
  o->apply_graph = 0;
  o->gemm_tile = 0;
  o->qr_single_launch = 1;
  o->hbm_budget_bytes = 0;
}

const char* spand_status_string(spand_status s) {
  switch (s) {
    case SPAND_OK: return "SPAND_OK";
    case SPAND_E_INVALID: return "SPAND_E_INVALID";
    case SPAND_E_NOT_SYMMETRIC: return "SPAND_E_NOT_SYMMETRIC";
    case SPAND_E_NOT_SPD: return "SPAND_E_NOT_SPD";
    case SPAND_E_NO_CONVERGENCE: return "SPAND_E_NO_CONVERGENCE";
    case SPAND_E_OOM: return "SPAND_E_OOM";
    case SPAND_E_HIP: return "SPAND_E_HIP";
    case SPAND_E_STATE: return "SPAND_E_STATE";
    case SPAND_E_LIMIT: return "SPAND_E_LIMIT";
  }
  return "unknown status";
}

spand_status spand_create(spand_ctx_t* out, int device, void* stream) {
  if (!out) return SPAND_E_INVALID;
  *out = nullptr;
  auto* ctx = new (std::nothrow) spand_ctx_s();
  if (!ctx) return SPAND_E_OOM;
  spand_status st = guarded(ctx, [&] {
    int ndev = 0;
    SPAND_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw spand::Error(SPAND_E_INVALID, "bad device ordinal");
    SPAND_HIP(hipSetDevice(device));
    ctx->c.device = device;
    ctx->c.pool = std::make_shared<spand::MemPool>(device, kPoolIdleBytes);
    ctx->vtmp[0].pool = ctx->vtmp[1].pool = ctx->c.pool;
    ctx->c.noalloc = spand::noalloc_scratch(device);
    if (stream) {
      ctx->c.stream = static_cast<hipStream_t>(stream);
    } else {
      SPAND_HIP(hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking));
      ctx->c.own_stream = true;
    }
  });
  if (st != SPAND_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return SPAND_OK;
}

void spand_destroy(spand_ctx_t ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
  if (ctx->c.own_stream) (void)hipStreamDestroy(ctx->c.stream);
  delete ctx;
}

const char* spand_last_error(spand_ctx_t ctx) { return ctx ? ctx->c.last_error.c_str() : ""; }

spand_status spand_analyze(spand_ctx_t ctx, int64_t n, const int64_t* rowptr, const int32_t* colind,
                           const double* coords, int32_t dim, const spand_opts* opts,
                           spand_plan_t* out) {
  if (!out) return SPAND_E_INVALID;
  *out = nullptr;
  auto plan = std::make_unique<spand_plan_s>();
  plan->id = g_plan_ids.fetch_add(1);
  spand_status st = guarded(ctx, [&] {
    using spand::Error;
    check_opts(opts);
    if (n <= 0 || !rowptr || !colind || (coords ? (dim < 1 || dim > 3) : dim != 0))
      throw Error(SPAND_E_INVALID, "bad matrix or coordinates");
    if (rowptr[0] != 0 || rowptr[n] < 0) throw Error(SPAND_E_INVALID, "bad rowptr");
    if (n >= (int64_t(1) << 31)) throw Error(SPAND_E_LIMIT, "n must be < 2^31");
    int depth = opts->depth;
    if (depth <= 0) depth = std::max(0, (int)std::lround(std::log2((double)n / 64.0)));
    if (depth > 40) throw Error(SPAND_E_INVALID, "depth too large");
    spand::Plan& P = plan->p;
    P.n = n;
    std::vector<double> gc;
    if (!coords) {   // coordinate-free: landmark distances in the graph of A
      gc = spand::graph_coords(n, rowptr, colind);
      coords = gc.data();
      dim = 3;
    }
    spand::analyze_plan(P, rowptr, colind, coords, dim, depth, opts->skip);
    spand::build_leaf_map(P);
  });
  if (st == SPAND_OK) *out = plan.release();
  return st;
}

spand_status spand_analyze_batch(spand_ctx_t ctx, int32_t count, const int64_t* n,
                                 const int64_t* const* rowptr, const int32_t* const* colind,
                                 const double* const* coords, const int32_t* dim,
                                 const int32_t* depth, const spand_opts* opts, spand_plan_t* out) {
  if (!out) return SPAND_E_INVALID;
  *out = nullptr;
  auto plan = std::make_unique<spand_plan_s>();
  plan->id = g_plan_ids.fetch_add(1);
  spand_status st = guarded(ctx, [&] {
    using spand::Error;
    check_opts(opts);
    if (count < 1 || !n || !rowptr || !colind || !coords || !dim)
      throw Error(SPAND_E_INVALID, "bad batch arguments");
    std::vector<spand::Plan> parts((size_t)count);   // sized once: plans are not moved
    std::vector<int> depths((size_t)count);
    for (int i = 0; i < count; ++i) {
      if (n[i] <= 0 || !rowptr[i] || !colind[i] ||
          (coords[i] ? (dim[i] < 1 || dim[i] > 3) : dim[i] != 0))
        throw Error(SPAND_E_INVALID, "bad matrix or coordinates of problem " + std::to_string(i));
      if (rowptr[i][0] != 0 || rowptr[i][n[i]] < 0)
        throw Error(SPAND_E_INVALID, "bad rowptr of problem " + std::to_string(i));
      int d = depth ? depth[i] : opts->depth;
      if (d <= 0) d = std::max(0, (int)std::lround(std::log2((double)n[i] / 64.0)));
      if (d > 40) throw Error(SPAND_E_INVALID, "depth too large");
      depths[i] = d;
      parts[i].n = n[i];
    }
    // the problems are analysed independently, on up to 16 host threads
    std::vector<std::exception_ptr> errs((size_t)count);
    std::atomic<int> next{0};
    auto run = [&] {
      for (int i; (i = next.fetch_add(1)) < count;) {
        try {
          std::vector<double> gc;
          const double* xy = coords[i];
          int d = dim[i];
          if (!xy) {
            gc = spand::graph_coords(n[i], rowptr[i], colind[i]);
            xy = gc.data();
            d = 3;
          }
          spand::analyze_plan(parts[i], rowptr[i], colind[i], xy, d, depths[i], opts->skip);
        } catch (...) {
          errs[i] = std::current_exception();
        }
      }
    };
    const int nth = std::min<int>({count, 16, (int)std::max(1u, std::thread::hardware_concurrency())});
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(run);
    run();
    for (auto& t : pool) t.join();
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
    spand::Plan& P = plan->p;
    std::vector<const spand::Plan*> pp;
    for (const spand::Plan& q : parts) pp.push_back(&q);
    spand::merge_plans(P, pp, opts->skip);
    spand::build_leaf_map(P);
  });
  if (st == SPAND_OK) *out = plan.release();
  return st;
}

spand_status spand_plan_segments(spand_plan_t plan, int32_t* count, int64_t* offsets) {
  if (!plan || !count) return SPAND_E_INVALID;
  const auto& so = plan->p.seg_off;
  *count = (int32_t)so.size() - 1;
  if (offsets) std::copy(so.begin(), so.end(), offsets);
  return SPAND_OK;
}

void spand_destroy_plan(spand_plan_t plan) { delete plan; }

spand_status spand_plan_sizes(spand_plan_t plan, int64_t* n, int64_t* nnz, int32_t* depth) {
  if (!plan) return SPAND_E_INVALID;
  if (n) *n = plan->p.n;
  if (nnz) *nnz = plan->p.nnz;
  if (depth) *depth = plan->p.depth;
  return SPAND_OK;
}

spand_status spand_plan_vertices(spand_plan_t plan, int32_t* lvl, int64_t* path, int64_t* perm) {
  if (!plan) return SPAND_E_INVALID;
  const spand::Plan& P = plan->p;
  if (lvl) std::memcpy(lvl, P.lvl.data(), P.n * sizeof(int32_t));
  if (path) std::memcpy(path, P.path.data(), P.n * sizeof(int64_t));
  if (perm) std::memcpy(perm, P.perm.data(), P.n * sizeof(int64_t));
  return SPAND_OK;
}

spand_status spand_plan_step_counts(spand_plan_t plan, int32_t l, int32_t* n_clusters,
                                    int32_t* n_interior, int64_t* n_adj, int64_t* n_child,
                                    int32_t* sparsified) {
  if (!plan || l < 0 || l > plan->p.depth) return SPAND_E_INVALID;
  const spand::StepPlan& st = plan->p.steps[l];
  if (n_clusters) *n_clusters = st.nc;
  if (n_interior) *n_interior = st.nI;
  if (n_adj) *n_adj = (int64_t)st.adj.size();
  if (n_child) *n_child = (int64_t)st.child.size();
  if (sparsified) *sparsified = st.sparsified ? 1 : 0;
  return SPAND_OK;
}

spand_status spand_plan_step_arrays(spand_plan_t plan, int32_t l, int64_t* key_lvl,
                                    int64_t* key_prefix, int64_t* adj_ptr, int32_t* adj,
                                    int32_t* colour, int64_t* child_ptr, int32_t* child) {
  if (!plan || l < 0 || l > plan->p.depth) return SPAND_E_INVALID;
  const spand::StepPlan& st = plan->p.steps[l];
  auto cp = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(key_lvl, st.key_lvl);
  cp(key_prefix, st.key_prefix);
  cp(adj_ptr, st.adj_ptr);
  cp(adj, st.adj);
  cp(colour, st.colour);
  if (child_ptr) {
    if (st.child_ptr.empty()) std::memset(child_ptr, 0, (st.nc + 1) * sizeof(int64_t));
    else cp(child_ptr, st.child_ptr);
  }
  cp(child, st.child);
  return SPAND_OK;
}

}  // extern "C"

namespace {

// Numeric factorization of plan P with the device values vals (nnz of P, in
// its CSR order) into a new core.
std::shared_ptr<FactorCore> factor_core(spand_ctx_t ctx, spand::Plan& P, const double* vals,
                                        const spand_opts* opts, bool copy_vals) {
  auto f = std::make_shared<FactorCore>();
  SPAND_HIP(hipSetDevice(ctx->c.device));
  f->device = ctx->c.device;
  upload_plan(P, ctx->c.device);
  const int64_t nnz = P.nnz;
  f->vals.pool = ctx->c.pool;
  f->d_vals = static_cast<double*>(f->vals.ensure(std::max<int64_t>(nnz, 1) * sizeof(double)));
  if (copy_vals)
    SPAND_HIP(hipMemcpyAsync(f->d_vals, vals, nnz * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->c.stream));
  // prescale: the factorization reads D^{-1/2} A D^{-1/2}; PCG keeps A
  const double* fvals = f->d_vals;
  spand::DevBuf svals;
  double* dsc = nullptr;
  if (opts->prescale) {
    const int64_t n = P.n;
    f->dscale.pool = ctx->c.pool;
    svals.pool = ctx->c.pool;
    dsc = static_cast<double*>(f->dscale.ensure(std::max<int64_t>(n, 1) * sizeof(double)));
    double* sv = static_cast<double*>(svals.ensure(std::max<int64_t>(nnz, 1) * sizeof(double)));
    int32_t* bad = static_cast<int32_t*>(ctx->c.ints.ensure(sizeof(int32_t)));
    spand::launch_prescale(P.d_rowptr, P.d_colind, f->d_vals, n, dsc, sv, bad, ctx->c.stream);
    int32_t hbad = 0;
    SPAND_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->c.stream));
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    if (hbad != INT32_MAX)
      throw spand::Error(SPAND_E_NOT_SPD, "prescale: diagonal entry of row " + std::to_string(hbad) +
                                              " is not positive");
    fvals = sv;
  }
  try {
    spand::run_factor(ctx->c, P, fvals, *opts, f->f);
  } catch (const spand::CoopPlacement&) {
    // a cooperative QR group was not on one XCD: redo with single-workgroup QRs
    std::fprintf(stderr, "spand: cooperative QR workgroups ran off their planned XCD; "
                         "factorization redone with single-workgroup QRs\n");
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    auto g = std::make_shared<FactorCore>();
    g->device = f->device;
    std::swap(g->vals.p, f->vals.p);
    std::swap(g->vals.bytes, f->vals.bytes);
    std::swap(g->vals.pool, f->vals.pool);
    std::swap(g->d_vals, f->d_vals);
    std::swap(g->dscale.p, f->dscale.p);
    std::swap(g->dscale.bytes, f->dscale.bytes);
    std::swap(g->dscale.pool, f->dscale.pool);
    f = std::move(g);
    spand_opts o2 = *opts;
    o2.qr_group = -1;
    spand::run_factor(ctx->c, P, fvals, o2, f->f);
    f->f.opts = *opts;
  }
  f->f.dscale = dsc;
  SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
  ctx->c.prof.resolve();
  f->f.stats.factor_bytes = (int64_t)f->f.arena.bytes_used();
  return f;
}

// Batch vectors for the handle of one problem: its n x nrhs columns embedded
// at its rows of an N x nrhs zero buffer (and copied back).
void embed(spand_ctx_t ctx, int slot, const spand_factor_s* h, int32_t nrhs, const double* x,
           double** X) {
  const int64_t N = h->core->f.plan->n;
  *X = static_cast<double*>(ctx->vtmp[slot].ensure(std::max<int64_t>(N * nrhs, 1) * sizeof(double)));
  SPAND_HIP(hipMemsetAsync(*X, 0, N * nrhs * sizeof(double), ctx->c.stream));
  if (x)
    SPAND_HIP(hipMemcpy2DAsync(*X + h->row0, N * sizeof(double), x, h->n * sizeof(double),
                               h->n * sizeof(double), nrhs, hipMemcpyDeviceToDevice, ctx->c.stream));
}
void extract(spand_ctx_t ctx, const spand_factor_s* h, int32_t nrhs, const double* X, double* y) {
  const int64_t N = h->core->f.plan->n;
  SPAND_HIP(hipMemcpy2DAsync(y, h->n * sizeof(double), X + h->row0, N * sizeof(double),
                             h->n * sizeof(double), nrhs, hipMemcpyDeviceToDevice, ctx->c.stream));
}

void check_ready(const spand_factor_s* f) {
  if (!f->core->f.prog) throw spand::Error(SPAND_E_STATE, "factor was stopped early (debug)");
}

}  // namespace

extern "C" {

spand_status spand_factor(spand_ctx_t ctx, spand_plan_t plan, const double* vals, const spand_opts* opts,
                          spand_factor_t* out) {
  if (!ctx || !plan || !out) return SPAND_E_INVALID;
  *out = nullptr;
  auto f = std::make_unique<spand_factor_s>();
  spand_status st = guarded(ctx, [&] {
    check_opts(opts);
    if (!vals) throw spand::Error(SPAND_E_INVALID, "vals is NULL");
    if (opts->skip != plan->p.skip)
      throw spand::Error(SPAND_E_INVALID, "skip differs from the one given to spand_analyze");
    f->core = factor_core(ctx, plan->p, vals, opts, true);
  });
  if (st == SPAND_OK) *out = f.release();
  return st;
}

spand_status spand_factor_batch(spand_ctx_t ctx, int32_t count, const spand_plan_t* plans,
                                const double* const* vals, const spand_opts* opts,
                                spand_factor_t* out) {
  if (!ctx || count < 1 || !plans || !vals || !out) return SPAND_E_INVALID;
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  std::vector<std::unique_ptr<spand_factor_s>> hs((size_t)count);
  spand_status st = guarded(ctx, [&] {
    using spand::Error;
    check_opts(opts);
    std::vector<uint64_t> key((size_t)count);
    for (int i = 0; i < count; ++i) {
      if (!plans[i] || !vals[i]) throw Error(SPAND_E_INVALID, "NULL plan or values of problem " + std::to_string(i));
      const spand::Plan& q = plans[i]->p;
      if (q.seg_off.size() != 2)
        throw Error(SPAND_E_INVALID, "problem " + std::to_string(i) + ": plan holds several problems");
      if (q.skip != opts->skip)
        throw Error(SPAND_E_INVALID, "problem " + std::to_string(i) + ": skip differs from opts");
      key[i] = plans[i]->id;
    }
    if (!ctx->batch_plan || ctx->batch_key != key) {
      auto M = std::make_shared<spand::Plan>();
      std::vector<const spand::Plan*> pp((size_t)count);
      for (int i = 0; i < count; ++i) pp[i] = &plans[i]->p;
      spand::merge_plans(*M, pp, opts->skip);
      spand::build_leaf_map(*M);
      ctx->batch_plan = std::move(M);
      ctx->batch_key = std::move(key);
    }
    std::shared_ptr<spand::Plan> M = ctx->batch_plan;
    SPAND_HIP(hipSetDevice(ctx->c.device));
    // the problems' values, concatenated on the device in the merged CSR order
    spand::DevBuf cat;
    cat.pool = ctx->c.pool;
    double* dv = static_cast<double*>(cat.ensure(std::max<int64_t>(M->nnz, 1) * sizeof(double)));
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
      const int64_t nz = plans[i]->p.nnz;
      SPAND_HIP(hipMemcpyAsync(dv + off, vals[i], nz * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->c.stream));
      off += nz;
    }
    std::shared_ptr<FactorCore> core = factor_core(ctx, *M, dv, opts, true);
    core->merged = M;
    for (int i = 0; i < count; ++i) {
      const spand::Plan& q = plans[i]->p;
      auto h = std::make_unique<spand_factor_s>();
      h->core = core;
      h->seg = i;
      h->n = q.n;
      h->row0 = M->seg_off[i];
      h->depth = q.depth;
      for (int l = 0; l <= q.depth; ++l) {
        h->nI.push_back(q.steps[l].nI);
        h->nc.push_back(q.steps[l].nc);
      }
      hs[i] = std::move(h);
    }
  });
  if (st == SPAND_OK)
    for (int i = 0; i < count; ++i) out[i] = hs[i].release();
  return st;
}

void spand_destroy_factor(spand_factor_t f) {
  if (!f) return;
  (void)hipSetDevice(f->core ? f->core->device : 0);
  delete f;
}

spand_status spand_factor_ranks(spand_factor_t f, int32_t l, int32_t* a, int32_t* k, int32_t* r,
                                int32_t* r2) {
  if (!f) return SPAND_E_INVALID;
  const spand::FactorObj& F = f->core->f;
  if (f->seg < 0) {
    if (l < 0 || l >= (int32_t)F.steps.size()) return SPAND_E_INVALID;
    const spand::StepRec& R = F.steps[l];
    const int nc = (int)R.r.size();
    for (int c = 0; c < nc; ++c) {
      const bool sp = R.r[c] >= 0;
      if (a) a[c] = sp ? R.n0[c] : -1;
      if (k) k[c] = R.k[c];
      if (r) r[c] = R.r[c];
      if (r2) r2[c] = R.r2[c];
    }
    return SPAND_OK;
  }
  // one problem of a batch: its own step l is batch step l + D - D_i, its
  // clusters sit at its offsets among the batch step's interiors and interfaces
  if (l < 0 || l > f->depth) return SPAND_E_INVALID;
  const int lm = l + (F.plan->depth - f->depth);
  const spand::StepRec& R = F.steps[lm];
  const spand::StepPlan& S = F.plan->steps[lm];
  const int own_nI = f->nI[l], own_nc = f->nc[l];
  for (int c = 0; c < own_nc; ++c) {
    const int x = c < own_nI ? S.seg_ioff[f->seg] + c : S.nI + S.seg_foff[f->seg] + (c - own_nI);
    const bool sp = R.r[x] >= 0;
    if (a) a[c] = sp ? R.n0[x] : -1;
    if (k) k[c] = R.k[x];
    if (r) r[c] = R.r[x];
    if (r2) r2[c] = R.r2[x];
  }
  return SPAND_OK;
}

spand_status spand_factor_info(spand_factor_t f, spand_factor_stats* st) {
  if (!f || !st) return SPAND_E_INVALID;
  *st = f->core->f.stats;
  return SPAND_OK;
}

spand_status spand_apply(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* x, double* y) {
  if (!ctx || !f || nrhs <= 0 || !x || !y) return SPAND_E_INVALID;
  return guarded(ctx, [&] {
    check_ready(f);
    SPAND_HIP(hipSetDevice(ctx->c.device));
    if (f->seg < 0) {
      spand::run_apply(ctx->c, f->F(), nrhs, x, y);
    } else {
      double* X = nullptr;
      embed(ctx, 0, f, nrhs, x, &X);
      spand::run_apply(ctx->c, f->F(), nrhs, X, X);
      extract(ctx, f, nrhs, X, y);
    }
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.prof.resolve();
  });
}

spand_status spand_apply_noalloc(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* x,
                                 double* y) {
  if (!ctx || !f || nrhs <= 0 || !x || !y) return SPAND_E_INVALID;
  return guarded(ctx, [&] {
    check_ready(f);
    if (f->seg >= 0)
      throw spand::Error(SPAND_E_INVALID, "allocation-free apply: a handle of a batch factor "
                                          "needs batch-sized vectors; use spand_apply");
    if (f->core->device != ctx->c.device)
      throw spand::Error(SPAND_E_INVALID, "factor lives on another device");
    SPAND_HIP(hipSetDevice(ctx->c.device));
    spand::run_apply_noalloc(ctx->c, f->F(), nrhs, x, y);
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.prof.resolve();
  });
}

spand_status spand_pcg(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* b, double* x,
                       double tol, int32_t maxit, int32_t* iters, double* relres) {
  if (!ctx || !f || nrhs <= 0 || !b || !x || !iters || !relres || maxit < 0 || !(tol > 0))
    return SPAND_E_INVALID;
  bool conv = false;
  spand_status st = guarded(ctx, [&] {
    check_ready(f);
    SPAND_HIP(hipSetDevice(ctx->c.device));
    if (f->seg < 0) {
      spand::run_pcg(ctx->c, f->F(), f->core->d_vals, nrhs, b, x, tol, maxit, iters, relres, &conv);
    } else {
      // the batch's segmented PCG with this problem's columns only (the
      // others' right-hand sides are zero, so their runs stop at once)
      const int nseg = (int)f->core->f.plan->seg_off.size() - 1;
      double *B = nullptr, *X = nullptr;
      embed(ctx, 0, f, nrhs, b, &B);
      embed(ctx, 1, f, nrhs, nullptr, &X);
      std::vector<int32_t> it((size_t)nseg * nrhs);
      std::vector<double> rr((size_t)nseg * nrhs);
      spand::run_pcg(ctx->c, f->F(), f->core->d_vals, nrhs, B, X, tol, maxit, it.data(), rr.data(),
                     &conv);
      extract(ctx, f, nrhs, X, x);
      for (int c = 0; c < nrhs; ++c) {
        iters[c] = it[(size_t)f->seg * nrhs + c];
        relres[c] = rr[(size_t)f->seg * nrhs + c];
      }
    }
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.prof.resolve();
  });
  if (st == SPAND_OK && !conv) {
    ctx->c.last_error = "PCG did not converge within maxit";
    return SPAND_E_NO_CONVERGENCE;
  }
  return st;
}

spand_status spand_pcg_batch(spand_ctx_t ctx, int32_t count, const spand_factor_t* factors,
                             const int32_t* nrhs, const double* const* b, double* const* x,
                             double tol, int32_t maxit, int32_t* iters, double* relres) {
  if (!ctx || count < 1 || !factors || !nrhs || !b || !x || !iters || !relres || maxit < 0 ||
      !(tol > 0))
    return SPAND_E_INVALID;
  bool all_conv = true;
  spand_status st = guarded(ctx, [&] {
    using spand::Error;
    std::vector<int64_t> col0((size_t)count + 1, 0);
    for (int i = 0; i < count; ++i) {
      if (!factors[i] || nrhs[i] < 1 || !b[i] || !x[i])
        throw Error(SPAND_E_INVALID, "bad factor or vectors of problem " + std::to_string(i));
      check_ready(factors[i]);
      col0[i + 1] = col0[i] + nrhs[i];
    }
    SPAND_HIP(hipSetDevice(ctx->c.device));
    std::vector<char> done((size_t)count, 0);
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      spand_factor_s* fi = factors[i];
      if (fi->seg < 0) {   // a plain factor: its own PCG
        bool conv = false;
        spand::run_pcg(ctx->c, fi->F(), fi->core->d_vals, nrhs[i], b[i], x[i], tol, maxit,
                       iters + col0[i], relres + col0[i], &conv);
        all_conv = all_conv && conv;
        done[i] = 1;
        continue;
      }
      // every handle of this batch core: one segmented PCG over the batch
      std::vector<int> members;
      int32_t w = 0;
      for (int j = i; j < count; ++j)
        if (!done[j] && factors[j]->core == fi->core) {
          members.push_back(j);
          w = std::max(w, nrhs[j]);
          done[j] = 1;
        }
      const int64_t N = fi->core->f.plan->n;
      const int nseg = (int)fi->core->f.plan->seg_off.size() - 1;
      double* B = static_cast<double*>(ctx->vtmp[0].ensure(std::max<int64_t>(N * w, 1) * sizeof(double)));
      double* X = static_cast<double*>(ctx->vtmp[1].ensure(std::max<int64_t>(N * w, 1) * sizeof(double)));
      SPAND_HIP(hipMemsetAsync(B, 0, N * w * sizeof(double), ctx->c.stream));
      for (int j : members) {
        const spand_factor_s* h = factors[j];
        SPAND_HIP(hipMemcpy2DAsync(B + h->row0, N * sizeof(double), b[j], h->n * sizeof(double),
                                   h->n * sizeof(double), nrhs[j], hipMemcpyDeviceToDevice,
                                   ctx->c.stream));
      }
      std::vector<int32_t> it((size_t)nseg * w);
      std::vector<double> rr((size_t)nseg * w);
      bool conv = false;
      spand::run_pcg(ctx->c, fi->F(), fi->core->d_vals, w, B, X, tol, maxit, it.data(), rr.data(),
                     &conv);
      all_conv = all_conv && conv;
      for (int j : members) {
        const spand_factor_s* h = factors[j];
        SPAND_HIP(hipMemcpy2DAsync(x[j], h->n * sizeof(double), X + h->row0, N * sizeof(double),
                                   h->n * sizeof(double), nrhs[j], hipMemcpyDeviceToDevice,
                                   ctx->c.stream));
        for (int c = 0; c < nrhs[j]; ++c) {
          iters[col0[j] + c] = it[(size_t)h->seg * w + c];
          relres[col0[j] + c] = rr[(size_t)h->seg * w + c];
        }
      }
    }
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.prof.resolve();
  });
  if (st == SPAND_OK && !all_conv) {
    ctx->c.last_error = "PCG did not converge within maxit";
    return SPAND_E_NO_CONVERGENCE;
  }
  return st;
}

spand_status spand_gemm_tuning(spand_ctx_t ctx, int32_t precision, int32_t* tiles, float* ms) {
  if (!ctx || precision < 0 || precision > 1) return SPAND_E_INVALID;
  const spand::GemmTuner& t = ctx->c.tuner;
  if (!t.tuned[precision]) return SPAND_E_STATE;
  for (int c = 0; c < spand::GemmTuner::kClasses; ++c) {
    if (tiles) tiles[c] = t.tile[precision][c];
    if (ms) {
      ms[2 * c] = t.ms[precision][c][0];
      ms[2 * c + 1] = t.ms[precision][c][1];
    }
  }
  return SPAND_OK;
}

spand_status spand_profile(spand_ctx_t ctx, int32_t enable) {
  if (!ctx) return SPAND_E_INVALID;
  return guarded(ctx, [&] {
    SPAND_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.prof.resolve();
    ctx->c.prof.on = enable != 0;
    ctx->c.prof.reset();
  });
}

spand_status spand_profile_only(spand_ctx_t ctx, const char* name) {
  if (!ctx) return SPAND_E_INVALID;
  ctx->c.prof.only = name ? name : "";
  return SPAND_OK;
}

spand_status spand_profile_entries(spand_ctx_t ctx, int32_t* count) {
  if (!ctx || !count) return SPAND_E_INVALID;
  *count = (int32_t)ctx->c.prof.entries.size();
  return SPAND_OK;
}

spand_status spand_profile_entry(spand_ctx_t ctx, int32_t i, char* name, int32_t name_len,
                                 double* ms, int64_t* calls, double* work) {
  if (!ctx || i < 0 || i >= (int32_t)ctx->c.prof.entries.size()) return SPAND_E_INVALID;
  const auto& e = ctx->c.prof.entries[i];
  if (name && name_len > 0) {
    std::strncpy(name, e.name.c_str(), name_len - 1);
    name[name_len - 1] = 0;
  }
  if (ms) *ms = e.ms;
  if (calls) *calls = e.calls;
  if (work) *work = e.work;
  return SPAND_OK;
}

spand_status spand_debug_block(spand_factor_t f, int32_t ci, int32_t cj, double* out, int32_t* rows,
                               int32_t* cols) {
  if (!f || f->seg >= 0 || f->core->f.stopped_at < 0 || !rows || !cols) return SPAND_E_STATE;
  const spand::FactorObj& F = f->core->f;
  const spand::StepPlan& st = F.plan->steps[F.stopped_at];
  if (ci < 0 || cj < 0 || ci >= st.nc || cj >= st.nc) return SPAND_E_INVALID;
  const int32_t* b = st.adj.data() + st.adj_ptr[ci];
  const int32_t* e = st.adj.data() + st.adj_ptr[ci + 1];
  const int32_t* it = std::lower_bound(b, e, cj);
  if (it == e || *it != cj) return SPAND_E_INVALID;
  const int64_t ee = st.adj_ptr[ci] + (it - b);
  const spand::PanelLayout& L = F.dbg_layout;
  *rows = F.dbg_ncur[ci];
  *cols = F.dbg_ncur[cj];
  if (out) {
    const double* src = F.dbg_panels.data() + L.off[ci] + L.coff[ee] * L.n[ci];
    for (int j = 0; j < *cols; ++j)
      for (int i = 0; i < *rows; ++i) out[i + (int64_t)j * *rows] = src[i + (int64_t)j * L.n[ci]];
  }
  return SPAND_OK;
}

}  // extern "C"
