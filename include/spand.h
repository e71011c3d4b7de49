/*
 * spand.h - C ABI of an MI355X implementation of spaND with first-order and
 * second-order sparsification (Klockiewicz, Cambier, Humble, Tchelepi, Darve,
 * "Second order accurate hierarchical approximate factorization of sparse SPD
 * matrices").
 *
 * Problem (Sec. 1): A x = b with A sparse symmetric positive definite (both
 * triangles stored, CSR) and one coordinate vector per row.  The library
 * computes the approximate factorization A ~ L L^T level by level (Alg. 2):
 * interiors of a nested-dissection level are eliminated by block Cholesky,
 * interfaces are scaled by the Cholesky factor of their diagonal block
 * (eq. prescale) and sparsified by an early-stopping column-pivoted QR at
 * tolerance eps (Alg. 1).  The preconditioner M = L^{-T} L^{-1} is applied in
 * PCG with a zero initial guess and a relative residual stop (Sec. 4).
 *
 * Conventions
 *  - Every call returns spand_status (0 = SPAND_OK, < 0 an error); no C++
 *    exception crosses the boundary.  spand_last_error() describes the last
 *    failure of a context, e.g. "interface block not SPD at step 7, cluster 12".
 *  - Host pointers are read during the call only and copied; the caller keeps
 *    ownership.  Device pointers (documented as such) must stay valid until the
 *    call returns; results written to device memory are complete when the call
 *    returns (the library synchronizes its stream before returning).
 *  - Plans and factors belong to the library until the matching destroy call.
 *  - One context per host thread.  The library allocates its device memory
 *    with hipMalloc on the context's device.
 */
#ifndef SPAND_H
#define SPAND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spand_ctx_s*    spand_ctx_t;
typedef struct spand_plan_s*   spand_plan_t;
typedef struct spand_factor_s* spand_factor_t;

typedef enum {
  SPAND_OK = 0,
  SPAND_E_INVALID = -1,        /* bad argument or option */
  SPAND_E_NOT_SYMMETRIC = -2,  /* pattern or values not symmetric */
  SPAND_E_NOT_SPD = -3,        /* a Cholesky factorization broke down */
  SPAND_E_NO_CONVERGENCE = -4, /* PCG hit maxit */
  SPAND_E_OOM = -5,            /* device allocation failed */
  SPAND_E_HIP = -6,            /* HIP runtime error */
  SPAND_E_STATE = -7,          /* call not valid in this state */
  SPAND_E_LIMIT = -8           /* a size exceeds a kernel limit */
} spand_status;

/* Sparsification schemes (Sec. 2): first order drops E and E^T (eq.
 * trailing-1); full second order keeps E in the outer factors and drops only
 * -E^T E (eq. trailing-2); superfine keeps E_2 only (eq. trailing-3). */
typedef enum { SPAND_FIRST_ORDER = 1, SPAND_SECOND_ORDER = 2, SPAND_SUPERFINE = 3 } spand_scheme;
/* Arithmetic of the factorization (a project addition; the paper's runs are
 * FP64).  SPAND_FP64: everything in FP64.  SPAND_FP32: the row panels, the
 * Schur and scaling products, the pivoted QR and the stored factor in FP32;
 * the diagonal-block Cholesky factorizations (and inverses) of the steps
 * l < top_fp64_levels (the top separator levels and the root) and of every
 * block above 64 rows are computed in FP64 and stored in FP32.
 * SPAND_FP32_BF16: as SPAND_FP32, with the Schur-complement products of the
 * interior elimination of the steps l >= top_fp64_levels on the BF16 matrix
 * cores (each FP32 operand split into two BF16 terms, three BF16 products per
 * pair), accumulated in FP32.  The apply keeps its vectors in FP64 (FP32
 * factor entries are widened on load), and PCG (SpMV, residuals, dot
 * products) is FP64 in every mode, so PCG refines the solution to the
 * requested tolerance whatever the precision. */
typedef enum { SPAND_FP64 = 0, SPAND_FP32 = 1, SPAND_FP32_BF16 = 2 } spand_precision;

typedef struct {
  int32_t depth;      /* nested-dissection depth D (levels D..0, Alg. 2); <= 0: round(log2(n/64)) */
  int32_t skip;       /* levels D..D-skip+1 neither scale nor sparsify (Sec. 4 skips 4) */
  double  eps;        /* 0 <= eps <= 1, RRQR tolerance (Alg. 1) */
  int32_t scheme;     /* spand_scheme */
  int32_t precision;  /* spand_precision */
  int32_t debug_stop_step;  /* >= 0: stop after sparsifying this step (parity dumps); -1: off */
  int32_t qr_group;     /* QR workgroups per interface: 0 auto, -1 single-workgroup kernel only,
                           g >= 1 force g (testing; capped by the coupling width and 32) */
  int32_t qr_list_cap;  /* tie candidates exchanged per workgroup: -1 default (32), 0..32 (testing) */
  int32_t qr_xcd_local; /* 1 (default); 0 treats every cooperative QR group as not placed on one
                           XCD, which makes the factorization fall back to the single-workgroup
                           QR (testing) */
  int32_t qr_lds_cols;  /* 0 (default): a cooperative QR workgroup keeps as many of its columns
                           in LDS as fit, the rest (interfaces wider than 32 workgroups' LDS)
                           in the row panel; c > 0: at most c in LDS (testing) */
  int32_t prescale;     /* 1: factor D^{-1/2} A D^{-1/2}, D = diag(A) (the symmetric diagonal
                           prescaling of the experiments, Sec. 4), and apply
                           M = D^{-1/2} M~ D^{-1/2} (M~ the preconditioner of the scaled matrix);
                           a non-positive diagonal entry gives SPAND_E_NOT_SPD.  0 (default): off */
  int32_t top_fp64_levels; /* FP32 precisions: the diagonal blocks of the steps l < top_fp64_levels
                              are factored in FP64 and their Schur products are FP32 (default 3:
                              the root and the two separator levels below it); ignored in FP64 */
  int32_t gemm_tile;    /* 0 (default): GEMM blocks of at most 32 x 32 on a one-wave-per-block
                           kernel, the others on the tile chosen per launch by the context's
                           autotuning; 64 or 128: that tile kernel for every block of every
                           GEMM launch (testing) */
  int32_t apply_graph;  /* 1: the factor's apply is captured in a HIP graph at its first use with a
                           given set of vector addresses and replayed afterwards (PCG applies
                           to the same buffers every iteration).  The caller must then not
                           allocate or free device memory from other threads while a PCG or
                           apply of this factor runs (those calls synchronize the device and
                           invalidate a capture).  0 (default): plain launches */
  int32_t qr_single_launch; /* 1 (default): the cooperative QR groups of one colour that need
                               several rounds of co-resident workgroups run in one launch, each
                               workgroup starting its group of the next round as soon as its
                               previous group is done; 0: one launch per round (testing) */
  int64_t hbm_budget_bytes; /* > 0: spand_factor fails with SPAND_E_OOM (and frees what it
                               allocated) as soon as the factor plus the working panels of a step
                               would hold more device memory than this; 0 (default): no limit */
} spand_opts;

void spand_default_opts(spand_opts* opts);
const char* spand_status_string(spand_status s);

/* Context: device ordinal and a HIP stream (hipStream_t passed as void*; NULL
 * = the library creates its own stream). */
spand_status spand_create(spand_ctx_t* out, int device, void* stream);
void spand_destroy(spand_ctx_t ctx);
const char* spand_last_error(spand_ctx_t ctx);

/* Symbolic analysis on the host: geometric nested dissection, clusters per
 * level, block structure with symbolic fill, interface colouring (Sec. 3,
 * Fig. 1; the coordinate-bisection partition replaces the algebraic spaND
 * partition, whose definition the paper defers to the base spaND paper).
 * rowptr[n+1], colind[nnz] (0-based, sorted or not), coords[n*dim] row-major:
 * host pointers.  coords = NULL with dim = 0 selects the coordinate-free
 * analysis: the bisection then runs on the hop distances of every vertex to
 * three landmark vertices of the graph of A (farthest-point sampling: the
 * vertex farthest from vertex 0, the one farthest from it, the one farthest
 * from both; lowest id on ties), so only the pattern is needed.
 * Checks pattern symmetry (SPAND_E_NOT_SYMMETRIC).  Pure host
 * work: ctx may be NULL (errors are then only reported by the status); the
 * plan is bound to a device by its first spand_factor. */
spand_status spand_analyze(spand_ctx_t ctx, int64_t n, const int64_t* rowptr, const int32_t* colind,
                           const double* coords, int32_t dim, const spand_opts* opts,
                           spand_plan_t* out);
/* Batch of independent problems (a block-diagonal system) analysed into one
 * plan, so that spand_factor, spand_apply and spand_pcg process all of them in
 * the same kernel launches (multi-problem batching, a project addition).
 * Problem i is given as for spand_analyze (n[i], rowptr[i], colind[i],
 * coords[i], dim[i]; host pointers, copied; coords[i] = NULL with dim[i] = 0
 * for the coordinate-free analysis); its rows follow those of problems
 * 0..i-1 in the batch numbering, and the batch's CSR values are the problems'
 * values concatenated in that order.  depth[i] (NULL: opts->depth, and <= 0
 * means round(log2(n[i]/64)) per problem) is each problem's own nested-
 * dissection depth; levels are aligned at the leaves, which keeps every
 * problem's own sparsified levels 1 <= l <= depth[i] - skip (Alg. 2, Sec. 4),
 * so each problem's factor is the one spand_analyze + spand_factor would give
 * it alone.  spand_pcg runs one CG per problem and column. */
spand_status spand_analyze_batch(spand_ctx_t ctx, int32_t count, const int64_t* n,
                                 const int64_t* const* rowptr, const int32_t* const* colind,
                                 const double* const* coords, const int32_t* dim,
                                 const int32_t* depth, const spand_opts* opts, spand_plan_t* out);
void spand_destroy_plan(spand_plan_t plan);
/* Problems of a plan (1 unless it came from spand_analyze_batch) and their row
 * offsets: offsets[count+1] (host, may be NULL to query the count). */
spand_status spand_plan_segments(spand_plan_t plan, int32_t* count, int64_t* offsets);

/* Plan queries (host arrays supplied by the caller, sized from the counts). */
spand_status spand_plan_sizes(spand_plan_t plan, int64_t* n, int64_t* nnz, int32_t* depth);
/* lvl[n], path[n], perm[n] (elimination permutation sorted by (D-lvl, path, id)) */
spand_status spand_plan_vertices(spand_plan_t plan, int32_t* lvl, int64_t* path, int64_t* perm);
/* counts of step l: clusters, interiors, adjacency entries, children entries */
spand_status spand_plan_step_counts(spand_plan_t plan, int32_t l, int32_t* n_clusters,
                                    int32_t* n_interior, int64_t* n_adj, int64_t* n_child,
                                    int32_t* sparsified);
/* arrays of step l: key_lvl[nc], key_prefix[nc], adj_ptr[nc+1], adj[n_adj] (sorted,
 * incl. self), colour[nc] (-1 interiors), child_ptr[nc+1], child[n_child]
 * (children in step l+1; empty at l = depth).  Any pointer may be NULL. */
spand_status spand_plan_step_arrays(spand_plan_t plan, int32_t l, int64_t* key_lvl,
                                    int64_t* key_prefix, int64_t* adj_ptr, int32_t* adj,
                                    int32_t* colour, int64_t* child_ptr, int32_t* child);

/* Numeric factorization on the device.  vals[nnz]: device pointer, values in
 * the CSR order given to spand_analyze.  SPAND_E_NOT_SPD names the step and
 * cluster of the first Cholesky breakdown. */
spand_status spand_factor(spand_ctx_t ctx, spand_plan_t plan, const double* vals, const spand_opts* opts,
                          spand_factor_t* out);
void spand_destroy_factor(spand_factor_t f);

/* Factorization of several separately analysed problems in the same kernel
 * launches (multi-problem batching, a project addition; each problem is
 * Alg. 2 on its own matrix, Sec. 1).  plans[count]: plans from spand_analyze
 * (one problem each, all with opts->skip); vals[count]: device pointers to
 * each problem's CSR values.  The plans are merged as spand_analyze_batch
 * would merge them (levels aligned at the leaves; the merged plan is cached
 * in the context for the next call with the same plans), the values are
 * concatenated on the device, and one factorization runs over all of them.
 * out[count] receives one factor handle per problem: every handle views the
 * same batch factor (released when its last handle is destroyed).  On a
 * handle, spand_factor_ranks reports that problem's own steps and clusters
 * (exactly what spand_factor gives it alone), spand_apply and spand_pcg take
 * that problem's own n x nrhs vectors (they run the whole batch's program with
 * the other problems' columns zero; use spand_pcg_batch to solve all problems
 * in one pass), and spand_factor_info reports the whole batch. */
spand_status spand_factor_batch(spand_ctx_t ctx, int32_t count, const spand_plan_t* plans,
                                const double* const* vals, const spand_opts* opts,
                                spand_factor_t* out);
/* PCG (Sec. 4) for several problems in one pass: factors[count] are handles
 * from spand_factor_batch (all from the same call) or plain factors; nrhs[i]
 * columns of b[i] / x[i] (device, n_i x nrhs[i] column-major) per problem.
 * Handles of one batch factor are solved together: one segmented PCG over the
 * batch (each (problem, column) an independent CG run, zero columns where a
 * problem has fewer right-hand sides than the widest); plain factors are
 * solved one after the other.  iters and relres (host) hold sum(nrhs)
 * entries, problem i's columns after those of problems 0..i-1.  Returns
 * SPAND_E_NO_CONVERGENCE if any run reaches maxit (results still written). */
spand_status spand_pcg_batch(spand_ctx_t ctx, int32_t count, const spand_factor_t* factors,
                             const int32_t* nrhs, const double* const* b, double* const* x,
                             double tol, int32_t maxit, int32_t* iters, double* relres);

/* Per-cluster sparsification record of step l: a (size before), k (coupling
 * width), r (eps rank), r2 (superfine rank, = r otherwise); -1 for interiors
 * and for steps that are not sparsified.  Host arrays of n_clusters. */
spand_status spand_factor_ranks(spand_factor_t f, int32_t l, int32_t* a, int32_t* k, int32_t* r,
                                int32_t* r2);
typedef struct {
  int64_t nnz_L;          /* memory metric numerator (Sec. 4): lower triangles of the L_s and
                             Z_p inverses, full G, the Householder vectors (a r - r(r-1)/2 plus
                             r tau), and the stored E part (second order) */
  double  flops;          /* algorithmic flops of the factorization */
  double  factor_seconds; /* wall time of spand_factor */
  int64_t factor_bytes;   /* device bytes held by the factor */
  int32_t root_size;
} spand_factor_stats;
spand_status spand_factor_info(spand_factor_t f, spand_factor_stats* st);

/* y = M x for nrhs columns; x, y: device pointers, n x nrhs column-major (any
 * nrhs: columns are processed in chunks that fit the kernels' LDS). */
spand_status spand_apply(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* x, double* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = M x as
 * spand_apply, on the same kernels, with every temporary in one fixed device
 * array of 64 MiB per device (SPAND_NOALLOC_SCRATCH_BYTES) that the library
 * holds from the first context on that device until the process ends.  Calls
 * no hipMalloc, hipFree or other allocating routine.  Columns are processed in
 * chunks that fit the array; SPAND_E_LIMIT if one column needs more scratch
 * than the array holds; SPAND_E_INVALID for a handle of a batch factor.  x, y:
 * device, n x nrhs column-major (may alias).  Every call on one device shares
 * that device's array (its contents are not kept from one call to the next),
 * so calls that overlap in time on one device, from different streams or
 * threads, race and give wrong results. */
#define SPAND_NOALLOC_SCRATCH_BYTES (64LL << 20)
spand_status spand_apply_noalloc(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* x,
                                 double* y);

/* PCG (Sec. 4): x0 = 0, stop when ||r_k||_2 < tol ||b||_2 per column and, for
 * a batch plan, per problem (each (problem, column) is an independent CG run);
 * b, x: device pointers (n x nrhs column-major); iters and relres (true
 * residual ||b - A x|| / ||b|| at exit): host arrays of segments x nrhs,
 * entry [s * nrhs + c] (segments = 1 for a single problem).  Returns
 * SPAND_E_NO_CONVERGENCE if a run reaches maxit. */
spand_status spand_pcg(spand_ctx_t ctx, spand_factor_t f, int32_t nrhs, const double* b, double* x,
                       double tol, int32_t maxit, int32_t* iters, double* relres);

/* Serving (a project addition around the method): a request loop on one
 * device.  Requests are solves A x = b with nrhs columns; a request names its
 * matrix by a caller-chosen key, and the first request with a key brings the
 * matrix (n, rowptr, colind, coords, dim, vals as for spand_analyze and
 * spand_factor, but vals is a HOST array; all copied at submit; later requests
 * with that key pass n = 0 or the same n and NULL matrix pointers).  `slots`
 * worker threads (1..16), each with its own context and stream, admit waiting
 * requests continuously: a slot takes up to max_batch of them, analyses and
 * factors the new matrices among them as one batch (spand_analyze_batch),
 * keeps those factors resident for later requests with the same keys, and
 * solves all its requests on one factor with one spand_pcg call (tol, maxit;
 * x0 = 0).  Factors whose device footprint would exceed max_bytes are not
 * admitted until least recently used idle factors have been released (their
 * host copies stay, and a later request re-factors); a single matrix larger
 * than the budget is admitted when nothing else is resident.  The result of a
 * request does not depend on the other requests it was batched with: each
 * problem's factor is the one spand_factor gives it alone, and each column is
 * its own CG run.  The slots' analyses, transfers, factorizations and PCG
 * solves overlap on the device; only the cooperative pivoted-QR launches of
 * the sparsified steps run one at a time per device (a lock the library holds
 * across every context of the process). */
typedef struct spand_server_s* spand_server_t;
spand_status spand_server_create(int32_t device, const spand_opts* opts, double tol, int32_t maxit,
                                 int64_t max_bytes, int32_t slots, int32_t max_batch,
                                 spand_server_t* out);
/* Queues a request; b: host, n x nrhs column-major (copied).  *req_id
 * receives its id.  SPAND_E_INVALID for a new key without its matrix or an n
 * that differs from the key's. */
spand_status spand_server_submit(spand_server_t srv, int64_t key, int64_t n, const int64_t* rowptr,
                                 const int32_t* colind, const double* coords, int32_t dim,
                                 const double* vals, int32_t nrhs, const double* b,
                                 int64_t* req_id);
/* Result of a request: wait = 1 blocks until it is done.  *done = 0: still
 * queued or running (nothing else written).  *done = 1: x (n x nrhs), iters
 * and relres (nrhs, as for spand_pcg) and latency (seconds from submit to
 * completion) are written (any may be NULL), the request is forgotten, and the
 * status is the request's own (SPAND_E_NO_CONVERGENCE if a column reached
 * maxit; x is still written then). */
spand_status spand_server_poll(spand_server_t srv, int64_t req_id, int32_t wait, int32_t* done,
                               double* x, int32_t* iters, double* relres, double* latency);
/* counters[9]: resident factor bytes, resident factors, queued requests,
 * factorization batches run, matrices factored, PCG calls, and microseconds
 * spent in analysis, factorization and PCG (wall time summed over slots). */
spand_status spand_server_stats(spand_server_t srv, int64_t* counters);
/* Last error message of a slot ("" if none). */
const char* spand_server_error(spand_server_t srv);
/* Finishes every queued request, then stops the slots and frees the factors. */
void spand_server_destroy(spand_server_t srv);

/* GEMM tile autotuning of a context (for reporting): the batched GEMM runs on
 * 64 x 64 or 128 x 128 output tiles; at its first factorization in a given
 * precision (FP64: precision 0; the FP32 forms: 1) a context times both on
 * synthetic batches of 64-, 128-, 256- and 512-row blocks and keeps the faster
 * per block-size class.  tiles[4] receives the chosen tile per class and
 * ms[8] the two trial times per class (NULL allowed); SPAND_E_STATE if the
 * context has not tuned that precision yet. */
spand_status spand_gemm_tuning(spand_ctx_t ctx, int32_t precision, int32_t* tiles, float* ms);

/* Per-kernel timing (for measurement).  spand_profile(ctx, 1) clears the
 * counters and starts recording a HIP event pair on the context stream around
 * every kernel launch of the library; spand_profile(ctx, 0) stops.  Entries
 * accumulate, per kernel name, the summed event time in ms, the number of
 * launches and (where the library knows it) the algorithmic work of those
 * launches: flops for k_cpqr / k_cpqr_coop (4(a-j)(k-j) per reflector j),
 * k_gemm (2 m n k per term; m (m + 1) k for a symmetric target of which only
 * the lower triangle is formed) and k_potrf_inv (n^3 / 3 per block), bytes
 * moved for k_copy, k_fill and k_scatter.  name receives at most name_len-1
 * characters. */
spand_status spand_profile(spand_ctx_t ctx, int32_t enable);
/* Restricts the timing to the launches of one kernel name (name = NULL or
 * "": every kernel), so that a timed run carries the event pairs of the
 * kernel it measures only. */
spand_status spand_profile_only(spand_ctx_t ctx, const char* name);
spand_status spand_profile_entries(spand_ctx_t ctx, int32_t* count);
spand_status spand_profile_entry(spand_ctx_t ctx, int32_t i, char* name, int32_t name_len,
                                 double* ms, int64_t* calls, double* work);

/* Debug dump for parity tests: with opts.debug_stop_step = l, after
 * spand_factor returns, copies block (ci, cj) of step l (after its
 * sparsification) to out (host, column-major, ld = *rows); rows/cols receive
 * the current block size.  out may be NULL to query the size. */
spand_status spand_debug_block(spand_factor_t f, int32_t ci, int32_t cj, double* out, int32_t* rows,
                               int32_t* cols);

#ifdef __cplusplus
}
#endif
#endif
