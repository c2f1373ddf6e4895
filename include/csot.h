/* csot.h -- C ABI of the cyclic-symmetric entropic optimal transport library (libcsot.so).
 *
 * The library implements, on one AMD MI355X (gfx950), the data-parallel path of the cyclic
 * Sinkhorn method of "Optimal Transport with Cyclic Symmetry" (Takeda, Akagi, Marumo, Niwa;
 * AAAI 2024) and plain full-size Sinkhorn beside it, plus the data-parallel steps of its
 * linear (unregularised) variant (Thm. 1) and its quadratically regularised variant (the
 * C-SROT algorithm).  Notation: the paper's vector length d, cyclic order n and regulariser
 * lambda are called n, K and eps here (lam for the quadratic regulariser); m = n / K.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Array arguments are DEVICE pointers unless marked [host].  Arrays are row-major and
 *   contiguous; points are block-major: point I = r*m + i is the i-th point of block r.
 *   Floating-point arrays are float32; scalars and statistics are float64.
 * - `stream` is a hipStream_t (NULL = the default stream).  Every call only enqueues work on
 *   it and returns, except where a [host] output is requested (the call then synchronises
 *   the stream) or `opts->validate` is set (it copies inputs to the host first).
 * - The library never allocates device memory.  Scratch space is the caller's `ws` buffer of
 *   `ws_bytes` bytes (256-byte aligned, at least ot_workspace_bytes()); its contents need no
 *   initialisation and are clobbered.  Two calls that share one `ws` must be ordered (same
 *   stream), and no state is kept between calls.
 * - Return value: OT_OK (0) or one of the OT_ERR_* codes below; ot_last_error() gives a
 *   message for the calling thread.  Arguments are validated on the host before any device
 *   work is enqueued, so an error return has enqueued nothing.  No C++ exception crosses the
 *   ABI and nothing aborts the process.
 */
#ifndef CSOT_H
#define CSOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OT_OK = 0,
  OT_ERR_ARG = 1,           /* null pointer, n % K != 0, bad dim, eps <= 0, ld too small ...  */
  OT_ERR_MASS = 2,          /* validate=1: negative/zero/non-finite marginal or |sum a - sum b| > 1e-6 */
  OT_ERR_NOT_SYMMETRIC = 3, /* validate=1: sampled cost entries are not block-circulant         */
  OT_ERR_NOCONV = 4,        /* max_iter reached before tol (only reported with host stats);
                               outputs and statistics are still valid                          */
  OT_ERR_NONFINITE = 5,     /* a potential became NaN/inf (only reported with host stats)       */
  OT_ERR_WORKSPACE = 6,     /* ws NULL or smaller than ot_workspace_bytes(), or misaligned      */
  OT_ERR_HIP = 7,           /* a HIP runtime call failed, or a device-side wait timed out       */
  OT_ERR_UNSUPPORTED = 8    /* size outside what the kernels are built for                      */
};

/* One transport problem (eq. problem_ROT of the paper under Assumption 1).
 *   dim in {2, 3}: costs are squared Euclidean distances C_IJ = |x_I - y_J|^2 recomputed
 *                  on the fly from the coordinates x, y ([n, dim] each); C must be NULL.
 *   dim == 0     : dense cost C [rows, ldc] with ldc >= n.  Calls on the reduced problem read
 *                  only block-row 0 (rows 0..m-1), whose column block k is the cost block
 *                  C_k of eq. blkstr_cost; full-size calls read all n rows.
 *   a, b         : marginals [n], positive; sum a == sum b (== 1 for probability vectors).
 *   eps          : the entropic regulariser lambda of eq. reg_for_entropy_ROT (> 0, absolute;
 *                  a caller wanting eps = factor * median(C) computes it itself).           */
typedef struct ot_problem {
  int32_t n, K, dim;
  const float* x;
  const float* y;
  const float* C;
  int64_t ldc;
  const float* a;
  const float* b;
  double eps;
} ot_problem;

/* Solver options; a NULL pointer means the defaults in brackets.
 *   tol        [1e-6]  stop when the full-space L2 row-marginal residual ||T 1 - a||_2 of the
 *                      current plan is <= tol (the column marginal is exact after each column
 *                      update).  tol = 0 runs exactly max_iter iterations.
 *   max_iter   [10000] >= 1.
 *   fold_fp64  [-1]    precision of the fold's log-sum over the K shifts.  1 or -1: costs,
 *                      their minimum and the shifted exponents in float64, the exponentials
 *                      of the shifted (non-positive) exponents in float32; logK is accurate
 *                      to float32 rounding at the speed of the float32 fold.  0: everything
 *                      in float32, whose error grows with C / eps.
 *   warm_start [0]     1: on entry g holds the initial column potential (natural units).
 *                      2 (ot_sinkhorn_full): on entry g[0..m) holds one block of a block-periodic
 *                      initial column potential, e.g. a reduced solution, and the solve starts
 *                      from it tiled K times (the second stage of Alg. 3); elsewhere as 1.
 *   validate   [0]     1: host-side checks of the marginals and of block-circulance (syncs).
 *   workgroups [0]     persistent solvers: number of cooperating workgroups (0 = automatic).
 *   timing_events [NULL]  host pointer to two hipEvent_t owned by the caller.  The persistent
 *                      solver calls (ot_sinkhorn_reduced, ot_sinkhorn_full,
 *                      ot_sinkhorn_reduced_batched) record the first on the stream immediately
 *                      before their solver kernel and the second right after it, so the elapsed
 *                      time between them is that kernel alone (no set-up, fold, values or
 *                      float64 check kernels).  Other calls ignore it.
 */
typedef struct ot_opts {
  double tol;
  int32_t max_iter;
  int32_t fold_fp64;
  int32_t warm_start;
  int32_t validate;
  int32_t workgroups;
  int32_t reserved;      /* must be 0 */
  void* timing_events;   /* hipEvent_t[2] or NULL */
} ot_opts;

/* [host] statistics of a solve.  err_row / err_col are recomputed in float64 on the GPU from
 * the returned potentials (full-space L2 norms, the marginal-error metric of Sec. 7.1). */
typedef struct ot_stats {
  int32_t iters;     /* completed (row, column) update pairs in the returned state            */
  int32_t converged; /* 1 when the float32 residual test met tol                               */
  double err_row;    /* ||T 1 - a||_2                                                          */
  double err_col;    /* ||T^T 1 - b||_2                                                        */
  double err_row32;  /* the float32 residual the stopping test used                            */
  int32_t flags;     /* bit 0: non-finite potential; bit 1: device wait timed out              */
  int32_t reserved;
} ot_stats;

/* Device-side statistics: solvers write OT_DSTATS_LEN doubles to `dstats` (device) in the
 * layout {iters, converged, err_row, err_col, err_row32, flags, redo, xcd_local}.  redo
 * (full-size solver only, else 0) counts the half-iterations of the first workgroup whose
 * shifted log-sum-exp had to be recomputed with a running maximum.  xcd_local (reduced solver
 * only, else 0) is 1 when all its workgroups ran on one XCD and exchanged potentials through
 * that XCD's L2. */
#define OT_DSTATS_LEN 8

/* Bytes of scratch space any call below needs for this problem and these options. */
size_t ot_workspace_bytes(const ot_problem* prob, const ot_opts* opts);

/* Fold (Alg. 2, first step; eq. def_Kij) and marginal fold (Alg. 3, stage 1).
 *   logK  [m, m] out: logK_ij = log sum_k exp(-C_ijk / eps), C_ijk = cost of block-row 0
 *         between point i and point k*m + j (C_k[i, j] of eq. blkstr_cost).
 *   alpha, beta [m] out: alpha_i = (1/K) sum_r a_{r m + i}; equal to the repeated block for
 *         periodic marginals (eq. assumption_for_input_vectors).
 * Errors: OT_ERR_ARG, OT_ERR_MASS / OT_ERR_NOT_SYMMETRIC (validate), OT_ERR_HIP. */
int ot_fold_kernel(const ot_problem* prob, const ot_opts* opts, float* logK, float* alpha,
                   float* beta, void* ws, size_t ws_bytes, void* stream);

/* Block-circulant projection of the cost of approximately symmetric data (the averaging of
 * Alg. 3, stage 1, applied to the cost as Lemma 1's proof averages a plan):
 *   Csym[i, k*m + j] = (1/K) sum_r C[r*m + i, ((r + k) mod K)*m + j],  Csym [m, ldcs], ldcs >= n.
 * The result is block-row 0 of a block-circulant cost; use it as a dense problem (dim = 0,
 * C = Csym, ldc = ldcs) for the reduced calls.  Errors: OT_ERR_ARG, OT_ERR_HIP. */
int ot_symmetrize_cost(const ot_problem* prob, float* Csym, int64_t ldcs, void* stream);

/* Cyclic Sinkhorn iterations on the folded m x m problem (Alg. 2; eq.
 * optimal_f_sinkhorn_logdomain and the log of eq. optimal_sinkhorn), in the log domain:
 *   f_i = eps log alpha_i - eps LSE_j(logK_ij + g_j / eps),
 *   g_j = eps log beta_j  - eps LSE_i(logK_ij + f_i / eps),
 * from g = 0 (q = 1) or the warm start, until the full-space row residual
 * sqrt(K) ||T_red 1 - alpha||_2 <= tol.  Only prob->n, K and eps are read.
 *   f, g [m] out (g is also the warm-start input); dstats [OT_DSTATS_LEN] device out or NULL;
 *   hstats [host] out or NULL (non-NULL synchronises and enables OT_ERR_NOCONV/NONFINITE).
 * One persistent launch (every workgroup resident at once, at most one per CU): workgroups
 * own row/column slabs of logK in LDS and exchange potentials through epoch-tagged slots in
 * device memory; no host round trip per iteration, and the launch can be captured in a graph.
 * Up to m = 2048 on a 256-CU device the slabs of one workgroup per CU are held in LDS; above,
 * padded copies of logK and its transpose are written to the workspace and read every
 * half-step (ot_workspace_bytes includes them for m > 1024).  Beyond m ~ 18900 even the staged
 * potentials exceed LDS and the call fails with OT_ERR_UNSUPPORTED. */
int ot_sinkhorn_reduced(const ot_problem* prob, const ot_opts* opts, const float* logK,
                        const float* alpha, const float* beta, float* f, float* g,
                        double* dstats, ot_stats* hstats, void* ws, size_t ws_bytes,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ot_sinkhorn_reduced with no workspace argument.
 * Same arguments, kernels and results otherwise.  Its scratch (the potential exchange slots
 * and residual partials) is a fixed array of OT_REDUCED_SCRATCH_BYTES in device memory, one
 * copy per device, held until the process ends; the call allocates nothing and calls no
 * allocating routine.  It covers every m whose slabs fit in LDS (up to m = 2048 on a 256-CU
 * device) and rejects, before any launch, a problem whose plan needs more scratch than the
 * array holds (m above that, or a workgroups hint that moves the slabs to device memory):
 * OT_ERR_UNSUPPORTED.  Runs on the current device; `stream` must belong to it.  The scratch
 * is cleared by a fill kernel at the start of every call, but every call on one device shares
 * it: calls that may overlap on one device (several streams, several host threads) race and
 * must be serialised by the caller.  Errors: as ot_sinkhorn_reduced, minus OT_ERR_WORKSPACE. */
#define OT_REDUCED_SCRATCH_BYTES (128u * 1024u)
int ot_sinkhorn_reduced_noalloc(const ot_problem* prob, const ot_opts* opts, const float* logK,
                                const float* alpha, const float* beta, float* f, float* g,
                                double* dstats, ot_stats* hstats, void* stream);

/* Plain full-size log-domain Sinkhorn on the n x n problem (Alg. 3, stage 2; the paper's
 * baseline), costs recomputed per tile from the coordinates (dim 2/3) or streamed from the
 * dense C (dim 0).  Same stopping rule, statistics and launch structure as the reduced call.
 * Workgroups (one per CU) own up to 4 blocks of at most 64 rows each, so n <= 256 x the CU
 * count (65536 on a 256-CU device); larger n fails with OT_ERR_UNSUPPORTED.
 *   f, g [n] out (g is also the warm-start input). */
int ot_sinkhorn_full(const ot_problem* prob, const ot_opts* opts, float* f, float* g,
                     double* dstats, ot_stats* hstats, void* ws, size_t ws_bytes,
                     void* stream);

/* [host] The launch configuration the persistent solvers would use for this problem and these
 * options on the current device (a query for tests and tuning; it enqueues nothing).
 *   ot_full_plan_info   info[6] = {workgroups, rows per row block, row blocks per workgroup,
 *                                  rows per lane RT, column split CQ, dense (dim 0)};
 *                       the variant (RT, CQ) is the full_solver_kernel instance launched.
 *   ot_reduced_plan_info info[6] = {workgroups, rows per workgroup, launch stride (8: all
 *                                  workgroups placed on one XCD), slabs in device memory,
 *                                  dynamic LDS bytes, threads per workgroup}.
 * Errors: OT_ERR_ARG (bad problem, options or NULL info), OT_ERR_UNSUPPORTED (no co-resident
 * configuration, or no device). */
int ot_full_plan_info(const ot_problem* prob, const ot_opts* opts, int32_t* info);
int ot_reduced_plan_info(const ot_problem* prob, const ot_opts* opts, int32_t* info);

/* Expansion of the reduced solution to the full block-circulant plan (Lemma 1, eq.
 * blkstr_optimal_solution; eq. optimality_condition; Alg. 2, last steps):
 *   T[r*m + i, c*m + j] = exp((f_i + g_j - C_{ij,(c - r) mod K}) / eps),  T [n, ldt], ldt >= n.
 * f, g [m] are reduced potentials.  Errors: OT_ERR_ARG, OT_ERR_HIP. */
int ot_expand_plan(const ot_problem* prob, const float* f, const float* g, float* T,
                   int64_t ldt, void* stream);

/* Cyclic linear OT (Thm. 1, eq. definition_G; Alg. 1, first step): for the unregularised
 * problem (eps is not used, but must be positive to pass validation), the min-fold of the cost
 * and the folded marginals:
 *   G[i, j] = min_k C_{ijk},  kmin[i, j] = the smallest k attaining it,  G, kmin [m, m];
 *   alpha_i = (1/K) sum_r a_{r m + i},  beta likewise,  [m].
 * Costs from coordinates are evaluated in float64 without fused multiply-adds (the same
 * arithmetic as a plain float64 evaluation, so ties and near-ties resolve identically); G is
 * stored in float32.  The small LP  min <G, S>, S 1 = alpha, S^T 1 = beta  (m^2 variables) is
 * the caller's: it is not data-parallel.  Errors: OT_ERR_ARG, OT_ERR_HIP. */
int ot_lot_fold(const ot_problem* prob, float* G, int32_t* kmin, float* alpha, float* beta,
                void* stream);

/* The full plan of the cyclic linear OT from the small LP's solution S [m, m] (eq.
 * optimal_solution_problem_CLOT placed by Lemma 1; Alg. 1, last steps):
 *   T[r*m + i, c*m + j] = S[i, j] if (c - r) mod K == kmin[i, j], else 0,  T [n, ldt], ldt >= n.
 * Its value <C, T> is K <G, S>, the optimum of the full problem when S is optimal.
 * Errors: OT_ERR_ARG, OT_ERR_HIP. */
int ot_lot_expand(const ot_problem* prob, const float* S, const int32_t* kmin, float* T,
                  int64_t ldt, void* stream);

/* Cyclic SROT with the quadratic regulariser phi(x) = (lam/2) x^2, x >= 0 (strongly convex; the
 * C-SROT section with Thm. 2, eq. dual_problem_cyclic_ROT): alternating maximisation of the
 * reduced dual over w, z [m] (in/out; zero-started unless opts->warm_start = 1).  An
 * iteration sets every w_i to the root of eq. derivative_of_objective_function,
 *   sum_{k,j} max(0, w_i + z_j - C_ijk) = lam alpha_i   (Newton on the piecewise linear sum),
 * then every z_j likewise; alpha, beta are the folded marginals.  The plan is
 * T_ijk = max(0, w_i + z_j - C_ijk) / lam (eq. optimality_condition), expanded by Lemma 1.
 * The iterations run in one persistent launch whose workgroups exchange the potentials
 * through device memory and test convergence on the device: with tol > 0 it stops after the
 * first iteration whose full-space row residual sqrt(K) ||T 1 - alpha||_2 (float64 sums) is at
 * most opts->tol; tol = 0 runs exactly max_iter iterations.  The float64 residuals are then
 * evaluated once and hstats [host, required] is filled by one copy at the end (the call
 * synchronises there, once).  With K = 1 and the full cost the same call solves the full-size
 * problem.  m is limited by the staged potential (about 16000 points); beyond it the call
 * fails with OT_ERR_UNSUPPORTED.  The workspace holds the folded marginals, the residuals,
 * the exchange slots and the statistics (ot_srot_workspace_bytes).  Errors: OT_ERR_ARG,
 * OT_ERR_WORKSPACE, OT_ERR_UNSUPPORTED, OT_ERR_NOCONV (outputs valid), OT_ERR_NONFINITE,
 * OT_ERR_HIP (also a timed-out exchange wait). */
size_t ot_srot_workspace_bytes(const ot_problem* prob);
int ot_srot_reduced(const ot_problem* prob, double lam, const ot_opts* opts, float* w, float* z,
                    ot_stats* hstats, void* ws, size_t ws_bytes, void* stream);

/* Objective values and gradients from converged potentials.
 *   reduced = 1: f, g [m] (plan T_ijk = exp((f_i + g_j - C_ijk)/eps) expanded by Lemma 1);
 *   reduced = 0: f, g [n] (plan T_IJ = exp((f_I + g_J - C_IJ)/eps)).
 *   out [8] device doubles: {P, D, <C,T>, err_row, err_col, mass, 0, 0} of the FULL problem:
 *     P = <C,T> + eps sum T (log T - 1)  (eq. problem_ROT with eq. reg_for_entropy_ROT),
 *         evaluated as sum T (C + eps (Z - 1)), Z = log T;  for reduced = 1 it is K times the
 *         reduced objective (eq. problem_CROT);
 *     D = <f,a> + <g,b> - eps sum T (eq. dual_problem_cyclic_ROT);
 *   dC   reduced: [m, lddc], lddc >= n, the derivative with respect to block-row 0 of the
 *        cost (the reduced problem's parameters; eq. problem_CROT): each entry C[i, k*m+j]
 *        appears in all K block-rows, so dC[i, k*m+j] = K T_ijk;
 *        full: [n, lddc], lddc >= n, dC = T;  NULL to skip.
 *   dx, dy [n, dim]: dP/dx_I = 2 sum_J T_IJ (x_I - y_J), dP/dy_J = 2 sum_I T_IJ (y_J - x_I);
 *        NULL to skip; must be NULL for dim = 0.
 *   da, db [n]: dP/da = f - mean(f), dP/db = g - mean(g) (tiled for reduced); NULL to skip.
 * The gradients are the envelope theorem applied to the dual (exact at the optimum).
 * Errors: OT_ERR_ARG, OT_ERR_WORKSPACE, OT_ERR_HIP. */
int ot_cost_and_grad(const ot_problem* prob, const float* f, const float* g, int32_t reduced,
                     double* out, float* dC, int64_t lddc, float* dx, float* dy, float* da,
                     float* db, void* ws, size_t ws_bytes, void* stream);

/* One problem of a batch.  The array of descriptors lives in DEVICE memory (all pointers in
 * it are device pointers); a host copy of the same array is given to ot_batched_plan.
 *   n, K, dim (2 or 3), eps   as in ot_problem; points and marginals x, y [n, dim], a, b [n];
 *   tile_cfg   two launch knobs the autotuner picks per (size bucket, K, dim): bits 0-7 the
 *              lanes cooperating on one row in the solve (16, 32, 64; 0 = by size), bits 8-15
 *              the fold's columns per tile in units of 64 (1 .. 16; 0 = 256);
 *   logK       scratch of 2 m mp + 2 m + 2 (2 mp + 64) floats, 16-byte aligned, mp = m
 *              rounded up to a multiple of 4 (folded kernel and its transpose with padded
 *              rows, folded marginals, then 2 mp + 64 64-bit exchange slots used when
 *              several workgroups solve the problem together);
 *   f, g [m]   out: reduced potentials (g is also the warm-start input);
 *   dx, dy [n, dim] out or NULL: gradients of the full objective with respect to every
 *              point, dP/dx_I = 2 sum_J T_IJ (x_I - y_J), dP/dy_J = 2 sum_I T_IJ (y_J - x_I),
 *              T the expanded plan (as ot_cost_and_grad with reduced potentials);
 *   out [8]    out: {P, D, <C,T>, err_row, err_col, iters, converged, flags} of the full
 *              problem, as ot_cost_and_grad and ot_stats define them;
 *   da, db [n] out or NULL: dP/da = f - mean(f), dP/db = g - mean(g), tiled over the blocks. */
typedef struct ot_batch_desc {
  int32_t n, K, dim, tile_cfg;
  double eps;
  const float* x;
  const float* y;
  const float* a;
  const float* b;
  float* logK;
  float* f;
  float* g;
  float* dx;
  float* dy;
  double* out;
  float* da;
  float* db;
} ot_batch_desc;

/* Number of int32 entries of a batch plan for `count` problems. */
size_t ot_batched_plan_len(int32_t count);

/* [host] Plan a batch: the work-queue order (largest problems first), the tile offsets of
 * the fold and value kernels and the solve tasks (problems above m = 256 are solved by a gang
 * of ceil(m / 128) workgroups, at most 32, that exchange potentials through the problem's
 * scratch).  `host_descs` is a host copy of the descriptor array; `plan`
 * [host] receives ot_batched_plan_len(count) int32 values that the caller copies to the
 * device.  Errors: OT_ERR_ARG (bad descriptor), OT_ERR_UNSUPPORTED (too many tiles). */
int ot_batched_plan(const ot_batch_desc* host_descs, int32_t count, int32_t* plan);

/* Scratch bytes of ot_sinkhorn_reduced_batched for `count` problems. */
size_t ot_batched_workspace_bytes(int32_t count);

/* Many independent cyclic problems of uneven size (the reduced path of Alg. 2 for each):
 * fold, cyclic Sinkhorn to tol (each problem stops on its own), objective values, float64
 * marginal errors and the gradients of every point (those outputs a descriptor leaves NULL
 * are skipped).  Launches on `stream`: two small clearing kernels (queue and accumulators), a
 * tiled fold, ONE persistent solve launch (one workgroup per CU, all resident) whose
 * workgroups pop tasks -- a whole small problem or one member's share of a large one -- from a
 * device work queue, one value/gradient launch per (dim, K) class of the batch (tiles of four
 * block-0 points; every plan entry T_ijk evaluated once per pass, the gradients of all K
 * copies of a point from float64 sums over the blocks) and a per-problem finalize.  No host
 * synchronisation, memset or allocation, so the call can be captured in a HIP graph.  `plan`
 * is the device copy of ot_batched_plan's output for the same descriptors and `plan_host`
 * [host] that output itself (launch sizes are read from it).  opts: tol, max_iter, fold_fp64,
 * warm_start and timing_events are honoured.  Errors: OT_ERR_ARG, OT_ERR_WORKSPACE, OT_ERR_HIP. */
int ot_sinkhorn_reduced_batched(const ot_batch_desc* descs, int32_t count, const int32_t* plan,
                                const int32_t* plan_host, const ot_opts* opts, void* ws,
                                size_t ws_bytes, void* stream);

/* Measurement, not a step of the method: the device's issue rates and latencies that the
 * roofline figures of the kernels above are quoted against.  Runs short micro-benchmark
 * kernels on `stream` and synchronises (not for graph capture).  out [host, OT_PEAKS_LEN]:
 *   [0] fp32 FMA issue rate (non-packed v_fma_f32), lane operations per second;
 *   [1] fp64 FMA issue rate;  [2] v_exp_f32 issue rate;
 *   [3] full-size Sinkhorn entries per second of its instruction mix (2 sub, 2 fma, exp2,
 *       add per entry on pre-scaled coordinates in registers): the ceiling of
 *       ot_sinkhorn_full;
 *   [4] device-to-device copy bandwidth, bytes read + written per second (256 MiB buffers);
 *   [5] one-way latency (s) of an epoch-tagged slot between two workgroups on one XCD with
 *       XCD-local publication (the reduced solver's exchange; NaN if a wait timed out);
 *   [6] the same between XCDs with device-scope publication;
 *   [7] 1 if [5] used XCD-local publication (both workgroups found on one XCD), else 0;
 *   [8] float64 matrix-core rate (v_mfma_f64_16x16x4f64), multiply-adds per second.
 * ws: ot_peaks_workspace_bytes() bytes, 256-byte aligned.  Errors: OT_ERR_ARG,
 * OT_ERR_WORKSPACE, OT_ERR_HIP. */
#define OT_PEAKS_LEN 9
size_t ot_peaks_workspace_bytes(void);
int ot_measure_peaks(double* out, void* ws, size_t ws_bytes, void* stream);

/* Message describing the last non-OK return on the calling thread ("" if none). */
const char* ot_last_error(void);

/* Library version string. */
const char* ot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSOT_H */
