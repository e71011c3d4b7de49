// Preconditioner apply y = M x, M = L^{-T} L^{-1} (Alg. 2 caption), and PCG
// (Sec. 4: zero initial guess, stop when ||r_k|| < tol ||b|| per column).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <string>

#include "apply.h"
#include "runtime.h"

namespace spand {

struct ApplyColour {
  ApSp* sp = nullptr;
  int32_t n_sp = 0, max_a = 0;
  ApWyTask* wyd = nullptr;   // wide WY apply: dots and update tasks
  ApWyTask* wyu = nullptr;
  int32_t n_wyd = 0, n_wyu = 0;
  int64_t usz = 0;           // u doubles per right-hand side
  ApEt* etf = nullptr;   // E tiles, forward
  ApEt* etb = nullptr;   // E tiles, backward
  int32_t n_etf = 0, n_etb = 0, max_nf = 0;
  ApGat* gat = nullptr;
  ApSrc* src = nullptr;
  int32_t n_gat = 0, max_n = 0;
};

struct ApplyStep {
  int l = 0;
  ApInt* in = nullptr;
  int32_t n_in = 0, max_in = 0;
  // large interiors: split GEMVs (forward rows + cols, backward rows + cols)
  bool split = false;
  ApMv* mv = nullptr;
  ApMvTask *f1 = nullptr, *f2 = nullptr, *b1 = nullptr, *b2 = nullptr;
  int32_t n_f1 = 0, n_f2 = 0, n_b1 = 0, n_b2 = 0;
  // interface scaling by split GEMVs: forward z = Zinv (gather result) rows;
  // backward Zinv^T z column dots into the scratch, then copied back
  bool ssplit = false;
  ApMv* smv = nullptr;
  ApMvTask *sf = nullptr, *sb1 = nullptr, *sb2 = nullptr;
  int32_t n_sf = 0, n_sb1 = 0, n_sb2 = 0;
  ApGat* gat = nullptr;
  ApSrc* src = nullptr;
  int32_t n_gat = 0, max_gat = 0;
  std::vector<ApplyColour> colours;
  ApScale* sc = nullptr;
  int32_t n_sc = 0, max_sc = 0;
};

// The launches of one apply (a fixed sequence for a factor, given the vector
// and scratch addresses and the column count) captured in a HIP graph: PCG
// applies the preconditioner to the same buffers every iteration, so the
// sequence is captured at the first application and replayed afterwards as one
// graph launch instead of a few hundred kernel launches.
struct ApplyGraph {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  const double* x = nullptr;
  double* y = nullptr;
  int32_t nrhs = 0;
  double *T = nullptr, *P = nullptr, *U = nullptr, *Y = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~ApplyGraph() { reset(); }
};

struct ApplyProg {
  std::vector<ApplyStep> steps;  // in forward order (depth ... 0)
  int64_t scratch = 0;           // doubles per right-hand side
  int64_t pscratch = 0;          // partial sums of the backward E tiles, per right-hand side
  int64_t uscratch = 0;          // u vectors of the wide WY apply, per right-hand side
  int64_t yscratch = 0;          // interior vectors of the split GEMVs, per right-hand side
  DevBuf T, P, U, Y;
  ApplyGraph graph;
};

FactorObj::~FactorObj() { delete prog; }



namespace {

int64_t find_adj(const StepPlan& st, int c, int target) {
  const int32_t* b = st.adj.data() + st.adj_ptr[c];
  const int32_t* e = st.adj.data() + st.adj_ptr[c + 1];
  const int32_t* it = std::lower_bound(b, e, target);
  if (it == e || *it != target) return -1;
  return st.adj_ptr[c] + (it - b);
}

}  // namespace

void begin_apply(FactorObj& F) {
  delete F.prog;
  F.prog = new ApplyProg();
  for (DevBuf* b : {&F.prog->T, &F.prog->P, &F.prog->U, &F.prog->Y}) b->pool = F.arena_pool;
}

// The apply program of step l (host descriptors written to the factor's
// mirrored metadata arena; flushed by finish_apply).  Steps are added in
// elimination order D ... 0, each once its factorization records are final,
// so this can run on a host thread beside the factorization of later steps.
void build_apply_step(FactorObj& F, int l) {
  const Plan& P = *F.plan;
  ApplyProg* prog = F.prog;
  const bool so = F.opts.scheme == SPAND_SECOND_ORDER;
  const bool sf = F.opts.scheme == SPAND_SUPERFINE;
  {
    const StepPlan& st = P.steps[l];
    const StepRec& R = F.steps[l];
    if (R.n0.empty()) return;  // stopped early
    ApplyStep as;
    as.l = l;
    const int nI = st.nI, nc = st.nc;
    std::vector<const int32_t*> dpos(nc, nullptr);
    {
      const int32_t* base = F.meta.upload(R.pos.idx);
      for (int c = 0; c < nc; ++c)
        if (R.pos.size(c) > 0) dpos[c] = base + R.pos.ptr[c];
    }
    // interiors
    std::vector<ApInt> ins;
    std::vector<int64_t> toff(nc, 0);
    int64_t tsz = 0;
    for (int sI = 0; sI < nI; ++sI) {
      const int n = R.n0[sI];
      if (n == 0) continue;
      std::vector<int32_t> nbr;
      for (int64_t e = st.adj_ptr[sI]; e < st.adj_ptr[sI + 1]; ++e) {
        const int w = st.adj[e];
        if (w == sI) continue;
        nbr.insert(nbr.end(), R.pos.begin(w), R.pos.begin(w) + R.pos.size(w));
      }
      ApInt d{};
      d.Linv = R.Linv[sI];
      d.G = R.G[sI];
      d.pos = dpos[sI];
      d.nbr_pos = F.meta.upload(nbr);
      d.toff = tsz;
      d.n = n;
      d.k = (int32_t)nbr.size();
      toff[sI] = tsz;
      tsz += d.k;
      ins.push_back(d);
      as.max_in = std::max(as.max_in, n);
    }
    prog->scratch = std::max(prog->scratch, tsz);
    as.in = F.meta.upload(ins);
    as.n_in = (int32_t)ins.size();
    if (as.n_in > 0 && as.n_in < kApSplitBelow) {
      // forward: y = L^-1 x (rows) into Y; t = G^T y (cols) into T, y back to z
      // backward: u = z - G z_W (rows) into Y; z = L^-T u (cols)
      std::vector<ApMv> mv;
      std::vector<ApMvTask> f1, f2, b1, b2;
      int64_t ysz = 0;
      for (const ApInt& d : ins) {
        const int32_t base = (int32_t)mv.size();
        ApMv m{};
        m.M = d.Linv; m.ld = d.n; m.rows = d.n; m.cols = d.n; m.tri = 1;
        m.xpos = d.pos; m.ooff = ysz; m.old = d.n;
        mv.push_back(m);                                            // base + 0: forward rows
        m = ApMv{};
        m.M = d.G; m.ld = d.n; m.rows = d.n; m.cols = d.k;
        m.xoff = ysz; m.xld = d.n; m.ooff = d.toff; m.old = d.k; m.wpos = d.pos;
        mv.push_back(m);                                            // base + 1: forward cols
        m = ApMv{};
        m.M = d.G; m.ld = d.n; m.rows = d.n; m.cols = d.k;
        m.xpos = d.nbr_pos; m.bpos = d.pos; m.ooff = ysz; m.old = d.n;
        mv.push_back(m);                                            // base + 2: backward rows
        m = ApMv{};
        m.M = d.Linv; m.ld = d.n; m.rows = d.n; m.cols = d.n; m.tri = 1;
        m.xoff = ysz; m.xld = d.n; m.opos = d.pos;
        mv.push_back(m);                                            // base + 3: backward cols
        for (int i0 = 0; i0 < d.n; i0 += kApMvRB) {
          f1.push_back({base + 0, i0});
          b1.push_back({base + 2, i0});
        }
        for (int c0 = 0; c0 == 0 || c0 < d.k; c0 += 4 * kApMvCB) f2.push_back({base + 1, c0});
        for (int c0 = 0; c0 < d.n; c0 += 4 * kApMvCB) b2.push_back({base + 3, c0});
        ysz += d.n;
      }
      as.split = true;
      as.mv = F.meta.upload(mv);
      as.f1 = F.meta.upload(f1);
      as.f2 = F.meta.upload(f2);
      as.b1 = F.meta.upload(b1);
      as.b2 = F.meta.upload(b2);
      as.n_f1 = (int32_t)f1.size();
      as.n_f2 = (int32_t)f2.size();
      as.n_b1 = (int32_t)b1.size();
      as.n_b2 = (int32_t)b2.size();
      prog->yscratch = std::max(prog->yscratch, ysz);
    }
    // interface gathers (+ scaling)
    std::vector<ApGat> gs;
    std::vector<ApSrc> srcs;
    std::vector<ApScale> scs;
    for (int w = nI; w < nc; ++w) {
      const int n = R.n0[w];
      if (n == 0) continue;
      ApGat g{};
      g.pos = dpos[w];
      g.Zinv = st.sparsified ? R.Zinv[w] : nullptr;
      g.src0 = (int64_t)srcs.size();
      for (int64_t e = st.adj_ptr[w]; e < st.adj_ptr[w + 1]; ++e) {
        const int sI = st.adj[e];
        if (sI >= nI) break;
        if (R.n0[sI] == 0) continue;
        const int64_t ee = find_adj(st, sI, w);
        // column of w inside G_s: sum of the sizes of s's earlier neighbours
        int32_t col = 0;
        for (int64_t q = st.adj_ptr[sI]; q < ee; ++q)
          if (st.adj[q] != sI) col += R.n0[st.adj[q]];
        srcs.push_back({toff[sI], col, R.kint[sI]});
      }
      g.src1 = (int64_t)srcs.size();
      g.n = n;
      if (g.src1 > g.src0 || g.Zinv) {
        gs.push_back(g);
        as.max_gat = std::max(as.max_gat, n);
      }
      if (st.sparsified) {
        scs.push_back({R.Zinv[w], dpos[w], n, 0});
        as.max_sc = std::max(as.max_sc, n);
      }
    }
    if (!scs.empty() && (int)scs.size() < kApSplitBelow) {
      std::vector<ApMv> mv;
      std::vector<ApMvTask> sf, sb1, sb2;
      int64_t ysz = 0;
      for (ApGat& g : gs) {
        if (!g.Zinv) continue;
        g.split = 1;
        g.yoff = ysz;
        ApMv m{};
        m.M = g.Zinv; m.ld = g.n; m.rows = g.n; m.cols = g.n; m.tri = 1;
        m.xoff = ysz; m.xld = g.n; m.opos = g.pos;
        const int32_t id = (int32_t)mv.size();
        mv.push_back(m);
        for (int i0 = 0; i0 < g.n; i0 += kApMvRB) sf.push_back({id, i0});
        ysz += g.n;
      }
      int64_t ysz2 = 0;
      for (const ApScale& c : scs) {
        ApMv m{};
        m.M = c.Zinv; m.ld = c.n; m.rows = c.n; m.cols = c.n; m.tri = 1;
        m.xpos = c.pos; m.ooff = ysz2; m.old = c.n;
        const int32_t id = (int32_t)mv.size();
        mv.push_back(m);
        for (int c0 = 0; c0 < c.n; c0 += 4 * kApMvCB) sb1.push_back({id, c0});
        m = ApMv{};
        m.rows = c.n; m.cols = 0; m.xoff = ysz2; m.xld = c.n; m.wpos = c.pos;
        sb2.push_back({(int32_t)mv.size(), 0});
        mv.push_back(m);
        ysz2 += c.n;
      }
      as.ssplit = true;
      as.smv = F.meta.upload(mv);
      as.sf = F.meta.upload(sf);
      as.sb1 = F.meta.upload(sb1);
      as.sb2 = F.meta.upload(sb2);
      as.n_sf = (int32_t)sf.size();
      as.n_sb1 = (int32_t)sb1.size();
      as.n_sb2 = (int32_t)sb2.size();
      prog->yscratch = std::max({prog->yscratch, ysz, ysz2});
    }
    as.gat = F.meta.upload(gs);
    as.src = F.meta.upload(srcs);
    as.n_gat = (int32_t)gs.size();
    as.sc = F.meta.upload(scs);
    as.n_sc = (int32_t)scs.size();
    // sparsification, per colour
    if (st.sparsified) {
      const int32_t* d_nbr_pos = F.meta.upload(R.sp_nbr_pos.idx);
      as.colours.resize(st.ncolours);
      for (int colour = 0; colour < st.ncolours; ++colour) {
        ApplyColour& ac = as.colours[colour];
        std::vector<ApSp> sps;
        std::vector<ApEt> etf, etb;
        std::vector<ApWyTask> wyd, wyu;
        int64_t csz = 0, psz = 0, usz = 0;
        std::vector<int64_t> ptoff(nc, -1);
        for (int p : st.order) {
          if (st.colour[p] != colour || R.n0[p] == 0) continue;
          ApSp d{};
          d.V = R.V[p];
          d.tau = R.tau[p];
          d.T = R.T[p];
          d.VT = R.VT[p];
          d.pos = dpos[p];
          d.nbr_pos = R.sp_nbr_pos.size(p) > 0 ? d_nbr_pos + R.sp_nbr_pos.ptr[p] : nullptr;
          d.a = R.n0[p];
          d.nref = R.r2[p];
          d.f0 = R.r[p];
          d.f1 = so ? R.n0[p] : (sf ? R.r2[p] : R.r[p]);
          d.k = R.k[p];
          d.lde = R.kmax[p];
          d.Et = (so || sf) && R.Y[p]
                     ? static_cast<const char*>(R.Y[p]) +
                           (F.f32 ? sizeof(float) : sizeof(double)) * (size_t)d.f0 * R.kmax[p]
                     : nullptr;
          d.toff = csz;
          ptoff[p] = csz;
          csz += d.k;
          const int nf = d.f1 - d.f0;
          d.part0 = psz;
          d.ntiles = 0;
          if (d.Et && nf > 0 && d.k > 0) {
            ApEt t{};
            t.Et = d.Et;
            t.lde = d.lde;
            t.nf = nf;
            t.k = d.k;
            for (int c0 = 0; c0 < d.k; c0 += kEtTileF) {
              t.c0 = c0;
              t.cn = std::min(kEtTileF, d.k - c0);
              t.pos = d.pos + d.f0;
              t.off = d.toff;
              etf.push_back(t);
            }
            for (int c0 = 0; c0 < d.k; c0 += kEtTileB) {
              t.c0 = c0;
              t.cn = std::min(kEtTileB, d.k - c0);
              t.pos = d.nbr_pos;
              t.off = psz;
              etb.push_back(t);
              psz += nf;
              ++d.ntiles;
            }
            ac.max_nf = std::max(ac.max_nf, nf);
          }
          d.uoff = usz;
          if (d.nref > 0) {
            const int32_t idx = (int32_t)sps.size();
            for (int j0 = 0; j0 < d.nref; j0 += kApWyCB) wyd.push_back({idx, j0});
            for (int i0 = 0; i0 < d.a; i0 += kApWyRB) wyu.push_back({idx, i0});
            usz += d.nref;
          }
          sps.push_back(d);
          ac.max_a = std::max(ac.max_a, d.a);
        }
        prog->scratch = std::max(prog->scratch, csz);
        prog->pscratch = std::max(prog->pscratch, psz);
        prog->uscratch = std::max(prog->uscratch, usz);
        ac.usz = usz;
        ac.wyd = F.meta.upload(wyd);
        ac.wyu = F.meta.upload(wyu);
        ac.n_wyd = (int32_t)wyd.size();
        ac.n_wyu = (int32_t)wyu.size();
        ac.sp = F.meta.upload(sps);
        ac.n_sp = (int32_t)sps.size();
        ac.etf = F.meta.upload(etf);
        ac.etb = F.meta.upload(etb);
        ac.n_etf = (int32_t)etf.size();
        ac.n_etb = (int32_t)etb.size();
        if (!(so || sf)) continue;
        // targets: interfaces adjacent to an interface of this colour
        std::vector<ApGat> eg;
        std::vector<ApSrc> es;
        for (int w = nI; w < nc; ++w) {
          if (st.colour[w] == colour) continue;
          const int wc = st.colour[w] < colour ? R.r[w] : R.n0[w];
          if (wc == 0) continue;
          ApGat g{};
          g.pos = dpos[w];
          g.src0 = (int64_t)es.size();
          for (int64_t e = st.adj_ptr[w]; e < st.adj_ptr[w + 1]; ++e) {
            const int p = st.adj[e];
            if (p < nI || st.colour[p] != colour || ptoff[p] < 0) continue;
            if (R.r[p] >= (so ? R.n0[p] : R.r2[p])) continue;  // no fine rows: E empty
            // offset of w inside W_p
            int32_t col = 0;
            for (int64_t q = st.adj_ptr[p]; q < st.adj_ptr[p + 1]; ++q) {
              const int x = st.adj[q];
              if (x == p || x < nI) continue;
              if (x == w) break;
              col += st.colour[x] < colour ? R.r[x] : R.n0[x];
            }
            es.push_back({ptoff[p], col, R.k[p]});
          }
          g.src1 = (int64_t)es.size();
          g.n = wc;
          if (g.src1 > g.src0) {
            eg.push_back(g);
            ac.max_n = std::max(ac.max_n, wc);
          }
        }
        ac.gat = F.meta.upload(eg);
        ac.src = F.meta.upload(es);
        ac.n_gat = (int32_t)eg.size();
      }
    }
    prog->steps.push_back(std::move(as));
  }
}

void finish_apply(Ctx& C, FactorObj& F) {
  F.meta.flush(C.stream);
  SPAND_HIP(hipStreamSynchronize(C.stream));
}


// LDS doubles the apply kernels stage for nrhs columns, at the largest
// cluster of each kernel class: interiors (x, y and the GEMV partial sums
// forward; y, u, partial sums and a gather chunk backward), interfaces (2
// vectors for the scaling; the WY apply; E tiles)
static int64_t apply_lds_need(const ApplyProg& pg, int32_t nrhs) {
  int64_t need = 0;
  for (const ApplyStep& as : pg.steps) {
    if (!as.split)
      need = std::max<int64_t>({need, (int64_t)as.max_in * (2 * nrhs + 4 * 4),
                                (int64_t)as.max_in * 6 * nrhs + 1024 * nrhs});
    need = std::max<int64_t>(need, (int64_t)(as.ssplit ? 0 : std::max(as.max_gat, 2 * as.max_sc)) * nrhs);
    for (const ApplyColour& ac : as.colours)
      need = std::max<int64_t>({need, (int64_t)ac.max_n * nrhs, (int64_t)ac.max_nf * nrhs + 2048,
                                (int64_t)kEtTileB * nrhs});
  }
  return need;
}

// scratch of one chunk of columns: the interiors' slices (T), the backward E
// partial sums (P), the WY u vectors (U) and the split-GEMV vectors (Y)
struct ApplyScratch {
  double *T, *P, *U, *Y;
};
static void apply_cols(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y,
                       const ApplyScratch& sc);

// columns per chunk that the apply kernels' LDS holds
static int32_t apply_lds_chunk(const ApplyProg& pg, int32_t nrhs) {
  constexpr int64_t kLds = 160 * 1024;
  int32_t chunk = 0;
  while (chunk < nrhs && apply_lds_need(pg, chunk + 1) * (int64_t)sizeof(double) <= kLds) ++chunk;
  if (chunk == 0) throw Error(SPAND_E_LIMIT, "cluster too large for the apply");
  return chunk;
}

// y = M x for nrhs columns (x and y may alias).  Columns are independent: they
// are processed in chunks of as many columns as the kernels' LDS holds.
void run_apply(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y) {
  ApplyProg& pg = *F.prog;
  const int32_t chunk = apply_lds_chunk(pg, nrhs);
  const int64_t n = F.plan->n;
  const int32_t w = std::min(chunk, nrhs);
  ApplyScratch sc;
  sc.T = static_cast<double*>(pg.T.ensure(std::max<int64_t>(pg.scratch, 1) * w * sizeof(double)));
  sc.P = static_cast<double*>(pg.P.ensure(std::max<int64_t>(pg.pscratch, 1) * w * sizeof(double)));
  sc.U = static_cast<double*>(pg.U.ensure(std::max<int64_t>(pg.uscratch, 1) * w * sizeof(double)));
  sc.Y = static_cast<double*>(pg.Y.ensure(std::max<int64_t>(pg.yscratch, 1) * w * sizeof(double)));
  auto launches = [&] {
    for (int32_t c0 = 0; c0 < nrhs; c0 += chunk)
      apply_cols(C, F, std::min(chunk, nrhs - c0), x + c0 * n, y + c0 * n, sc);
  };
  // per-kernel event timing of the apply's kernels needs the individual launches
  const bool timed = C.prof.on && (C.prof.only.empty() || C.prof.only.rfind("k_ap_", 0) == 0 ||
                                   C.prof.only == "k_copy_vec" || C.prof.only == "k_scale_vec");
  if (timed || !F.opts.apply_graph) {
    launches();
    return;
  }
  ApplyGraph& g = pg.graph;
  const bool same = g.exec && g.stream == C.stream && g.x == x && g.y == y && g.nrhs == nrhs &&
                    g.T == sc.T && g.P == sc.P && g.U == sc.U && g.Y == sc.Y;
  if (!same) {
    g.reset();
    // the descriptors the apply reads were uploaded when the factor was
    // finished; nothing is pending, so the capture holds kernel nodes only
    C.upload.flush(C.stream);
    SPAND_HIP(hipStreamBeginCapture(C.stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t graph = nullptr;
    try {
      launches();
    } catch (...) {
      (void)hipStreamEndCapture(C.stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    SPAND_HIP(hipStreamEndCapture(C.stream, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    SPAND_HIP(e);
    g.stream = C.stream;
    g.x = x;
    g.y = y;
    g.nrhs = nrhs;
    g.T = sc.T;
    g.P = sc.P;
    g.U = sc.U;
    g.Y = sc.Y;
  }
  SPAND_HIP(hipGraphLaunch(g.exec, C.stream));
}

// ---------------------------------------------------------------------------
// Allocation-free apply: the same kernels, with every temporary in one fixed
// device array per device (held until the process ends).  In host code
// `scratch` names a host-side stand-in, not device memory: its device address
// comes from hipGetSymbolAddress, taken once per device at context set-up.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

void* noalloc_scratch(int device) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) throw Error(SPAND_E_INVALID, "bad device ordinal");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[device]) {
    void* p = nullptr;   // the caller has made `device` current
    SPAND_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[device] = p;
  }
  return ptr[device];
}

void run_apply_noalloc(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y) {
  ApplyProg& pg = *F.prog;
  if (!C.noalloc) throw Error(SPAND_E_STATE, "no fixed scratch on this context's device");
  // doubles per column of each part, rounded up to 256 bytes
  auto up = [](int64_t v) { return (std::max<int64_t>(v, 1) + 31) / 32 * 32; };
  const int64_t pt = up(pg.scratch), pp = up(pg.pscratch), pu = up(pg.uscratch), py = up(pg.yscratch);
  const int64_t per = (pt + pp + pu + py) * (int64_t)sizeof(double);
  const int64_t fit = (int64_t)kNoAllocScratchBytes / per;
  if (fit < 1)
    throw Error(SPAND_E_LIMIT, "allocation-free apply: one column needs " + std::to_string(per) +
                                   " bytes of scratch, more than the fixed " +
                                   std::to_string(kNoAllocScratchBytes) + " bytes");
  const int32_t chunk = (int32_t)std::min<int64_t>(apply_lds_chunk(pg, nrhs), fit);
  double* base = static_cast<double*>(C.noalloc);
  ApplyScratch sc;
  sc.T = base;
  sc.P = sc.T + pt * chunk;
  sc.U = sc.P + pp * chunk;
  sc.Y = sc.U + pu * chunk;
  const int64_t n = F.plan->n;
  for (int32_t c0 = 0; c0 < nrhs; c0 += chunk)
    apply_cols(C, F, std::min(chunk, nrhs - c0), x + c0 * n, y + c0 * n, sc);
}

static void apply_cols(Ctx& C, FactorObj& F, int32_t nrhs, const double* x, double* y,
                       const ApplyScratch& sc) {
  hipStream_t s = C.stream;
  const int64_t n = F.plan->n;
  ApplyProg& pg = *F.prog;
  const bool f32 = F.f32;
  double* T = sc.T;
  double* Pp = sc.P;
  double* U = sc.U;
  double* Ys = sc.Y;
  if (F.dscale) SPAND_PROF(C, "k_scale_vec", launch_scale_vec(x, F.dscale, y, n, nrhs, s));
  else if (x != y) SPAND_PROF(C, "k_copy_vec", launch_copy_vec(x, y, n * nrhs, s));
  for (const ApplyStep& as : pg.steps) {
    if (as.split) {
      SPAND_PROF(C, "k_ap_mv_rows", launch_ap_mv_rows(as.f1, as.n_f1, as.mv, y, n, nrhs, nullptr, Ys, f32, s));
      SPAND_PROF(C, "k_ap_mv_cols", launch_ap_mv_cols(as.f2, as.n_f2, as.mv, y, n, nrhs, Ys, T, f32, s));
    } else {
      SPAND_PROF(C, "k_ap_int_fwd", launch_ap_int_fwd(as.in, as.n_in, y, n, nrhs, T, as.max_in, f32, s));
    }
    SPAND_PROF(C, "k_ap_gather", launch_ap_gather(as.gat, as.src, as.n_gat, y, n, nrhs, T,
                                                  as.ssplit ? 0 : as.max_gat, f32, s, Ys));
    if (as.ssplit)
      SPAND_PROF(C, "k_ap_mv_rows", launch_ap_mv_rows(as.sf, as.n_sf, as.smv, y, n, nrhs, Ys, nullptr, f32, s));
    for (const ApplyColour& ac : as.colours) {
      SPAND_PROF(C, "k_ap_wy_dots", launch_ap_wy_dots(ac.wyd, ac.n_wyd, ac.sp, y, n, nrhs, nullptr,
                                                      U, ac.usz, 1, f32, s));
      SPAND_PROF(C, "k_ap_wy_update", launch_ap_wy_update(ac.wyu, ac.n_wyu, ac.sp, y, n, nrhs,
                                                          nullptr, U, ac.usz, 1, f32, s));
      SPAND_PROF(C, "k_ap_et_fwd", launch_ap_et_fwd(ac.etf, ac.n_etf, y, n, nrhs, T, ac.max_nf, f32, s));
      SPAND_PROF(C, "k_ap_gather", launch_ap_gather(ac.gat, ac.src, ac.n_gat, y, n, nrhs, T, ac.max_n, f32, s));
    }
  }
  for (auto it = pg.steps.rbegin(); it != pg.steps.rend(); ++it) {
    const ApplyStep& as = *it;
    for (auto c = as.colours.rbegin(); c != as.colours.rend(); ++c) {
      SPAND_PROF(C, "k_ap_et_bwd", launch_ap_et_bwd(c->etb, c->n_etb, y, n, nrhs, Pp, f32, s));
      SPAND_PROF(C, "k_ap_wy_dots", launch_ap_wy_dots(c->wyd, c->n_wyd, c->sp, y, n, nrhs, Pp, U,
                                                      c->usz, 0, f32, s));
      SPAND_PROF(C, "k_ap_wy_update", launch_ap_wy_update(c->wyu, c->n_wyu, c->sp, y, n, nrhs, Pp,
                                                          U, c->usz, 0, f32, s));
    }
    if (as.ssplit) {
      SPAND_PROF(C, "k_ap_mv_cols", launch_ap_mv_cols(as.sb1, as.n_sb1, as.smv, y, n, nrhs, nullptr, Ys, f32, s));
      SPAND_PROF(C, "k_ap_mv_cols", launch_ap_mv_cols(as.sb2, as.n_sb2, as.smv, y, n, nrhs, Ys, nullptr, f32, s));
    } else {
      SPAND_PROF(C, "k_ap_scale_bwd", launch_ap_scale_bwd(as.sc, as.n_sc, y, n, nrhs, as.max_sc, f32, s));
    }
    if (as.split) {
      SPAND_PROF(C, "k_ap_mv_rows", launch_ap_mv_rows(as.b1, as.n_b1, as.mv, y, n, nrhs, nullptr, Ys, f32, s));
      SPAND_PROF(C, "k_ap_mv_cols", launch_ap_mv_cols(as.b2, as.n_b2, as.mv, y, n, nrhs, Ys, nullptr, f32, s));
    } else {
      SPAND_PROF(C, "k_ap_int_bwd", launch_ap_int_bwd(as.in, as.n_in, y, n, nrhs, as.max_in, f32, s));
    }
  }
  if (F.dscale) SPAND_PROF(C, "k_scale_vec", launch_scale_vec(y, F.dscale, y, n, nrhs, s));
}

void run_pcg(Ctx& C, FactorObj& F, const double* d_vals, int32_t nrhs, const double* b, double* x,
             double tol, int32_t maxit, int32_t* iters, double* relres, bool* converged) {
  // one CG run per (segment, column): the segments are the independent
  // problems of a batch plan (one segment otherwise)
  hipStream_t s = C.stream;
  const Plan& P = *F.plan;
  const int64_t n = P.n;
  const int64_t nv = n * nrhs;
  const int32_t nseg = (int32_t)P.seg_off.size() - 1;
  const int32_t ne = nseg * nrhs;
  const int32_t* seg_id = nseg > 1 ? P.d_seg_id : nullptr;
  DevArena work;
  work.set_pool(C.pool);
  double* r = work.alloc_n<double>(nv);
  double* z = work.alloc_n<double>(nv);
  double* p = work.alloc_n<double>(nv);
  double* q = work.alloc_n<double>(nv);
  double* partial = work.alloc_n<double>((size_t)dot_blocks(nseg) * ne);
  double* sc = work.alloc_n<double>(4 * (size_t)ne);  // rho | rho_new | pq | rr
  double* rho = sc;
  double* rho_new = sc + ne;
  double* pq = sc + 2 * ne;
  double* rr = sc + 3 * ne;
  int32_t* active = work.alloc_n<int32_t>(ne);
  std::vector<int32_t> h_active(ne, 1);
  std::vector<double> h_bn(ne), h_rr(ne);

  SPAND_PROF(C, "k_dot", launch_dot(b, b, n, nrhs, P.d_seg_off, nseg, partial, rr, s));
  SPAND_HIP(hipMemcpyAsync(h_bn.data(), rr, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  SPAND_HIP(hipStreamSynchronize(s));
  for (int e = 0; e < ne; ++e) {
    h_bn[e] = std::sqrt(h_bn[e]);
    iters[e] = 0;
    if (h_bn[e] == 0.0) h_active[e] = 0;
  }
  SPAND_HIP(hipMemsetAsync(x, 0, nv * sizeof(double), s));
  SPAND_HIP(hipMemcpyAsync(active, h_active.data(), ne * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SPAND_PROF(C, "k_copy_vec", launch_copy_vec(b, r, nv, s));
  run_apply(C, F, nrhs, r, z);
  SPAND_PROF(C, "k_dot", launch_dot(r, z, n, nrhs, P.d_seg_off, nseg, partial, rho_new, s));
  SPAND_PROF(C, "k_pcg_p",
             launch_pcg_p(p, z, rho, rho_new, active, seg_id, n, nrhs, nseg, 1, s));
  int nact = 0;
  for (int e = 0; e < ne; ++e) nact += h_active[e];
  for (int it = 1; it <= maxit && nact > 0; ++it) {
    SPAND_PROF(C, "k_spmv", launch_spmv(P.d_rowptr, P.d_colind, d_vals, n, nrhs, p, q, s));
    SPAND_PROF(C, "k_dot", launch_dot(p, q, n, nrhs, P.d_seg_off, nseg, partial, pq, s));
    SPAND_PROF(C, "k_pcg_xr", launch_pcg_xr(x, r, p, q, rho, pq, active, seg_id, n, nrhs, s));
    SPAND_PROF(C, "k_dot", launch_dot(r, r, n, nrhs, P.d_seg_off, nseg, partial, rr, s));
    SPAND_HIP(hipMemcpyAsync(h_rr.data(), rr, ne * sizeof(double), hipMemcpyDeviceToHost, s));
    SPAND_HIP(hipStreamSynchronize(s));
    bool changed = false;
    for (int e = 0; e < ne; ++e)
      if (h_active[e] && std::sqrt(h_rr[e]) < tol * h_bn[e]) {
        h_active[e] = 0;
        iters[e] = it;
        --nact;
        changed = true;
      } else if (h_active[e]) {
        iters[e] = it;
      }
    if (nact == 0) break;
    if (changed)
      SPAND_HIP(hipMemcpyAsync(active, h_active.data(), ne * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
    run_apply(C, F, nrhs, r, z);
    SPAND_PROF(C, "k_dot", launch_dot(r, z, n, nrhs, P.d_seg_off, nseg, partial, rho_new, s));
    SPAND_PROF(C, "k_pcg_p",
               launch_pcg_p(p, z, rho, rho_new, active, seg_id, n, nrhs, nseg, 0, s));
  }
  // true residual
  SPAND_PROF(C, "k_spmv", launch_spmv(P.d_rowptr, P.d_colind, d_vals, n, nrhs, x, q, s));
  SPAND_PROF(C, "k_residual", launch_residual(b, q, n, nrhs, s));
  SPAND_PROF(C, "k_dot", launch_dot(q, q, n, nrhs, P.d_seg_off, nseg, partial, rr, s));
  SPAND_HIP(hipMemcpyAsync(h_rr.data(), rr, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  SPAND_HIP(hipStreamSynchronize(s));
  *converged = nact == 0;
  for (int e = 0; e < ne; ++e) relres[e] = h_bn[e] > 0 ? std::sqrt(h_rr[e]) / h_bn[e] : 0.0;
}

}  // namespace spand
