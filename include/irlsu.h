/*
 * irlsu -- IRLS + PCG weighted-L1 phase unwrapping on AMD Instinct MI355X.
 *
 * C ABI of the library.  Plain pointers and sizes only; every pointer named
 * "device" is HIP device memory, every other pointer is host memory.  No
 * function throws; every function returns an irlsu_status.  All work is
 * enqueued on the caller's HIP stream (passed as void*, a hipStream_t; NULL
 * is the default stream) and is asynchronous unless stated otherwise.
 *
 * The method (paper: Dubois-Taine, Akiki, d'Aspremont, "Iteratively
 * Reweighted Least Squares for Phase Unwrapping", arXiv 2401.09961):
 *
 *   minimise over mean-zero U   sum C^v |S U - G^v| + sum C^h |U T - G^h|
 *
 * (Section 2, problem (prob:main-matrix-form)), with G the wrapped phase
 * differences of the observed phase X and C > 0 per-edge weights.  The
 * library runs the slack-eliminated form of the paper's IRLS (Algorithm 1):
 * eliminating V^v, V^h from the linear system of Proposition 1 leaves the
 * weighted 5-point system D^T Omega D U = D^T Omega G, here with IRLS weights
 * Omega = C / max(|DU - G|, eps), which minimises sum C h_eps(DU - G) (the
 * Huber function, the Moreau envelope that the paper's penalty produces).
 * Each system is solved by preconditioned CG (Algorithm 2) with the U block
 * of the block-diagonal preconditioner of Section 3.3: the Neumann
 * Laplacian, inverted through its eigendecomposition -- the dense products
 * P_S^T R P_T and P_S Z' P_T^T of Section 3.3, where P is the orthonormal
 * DCT-II basis -- with the zero mode removed (Appendix B).
 *
 * Internal layout.  Step-level entry points take images in the plan's
 * internal layout: Np rows by ld columns, row-major, columns contiguous,
 * with Np >= N and ld >= M padded to the plan's tile size (irlsu_plan_info).
 * Pixel (i, j) is element i * ld + j.  Vertical edge (i, j) joins pixels
 * (i, j) and (i+1, j); horizontal edge (i, j) joins (i, j) and (i, j+1).
 * Edge arrays use the same Np x ld shape; entries of edges that do not exist
 * (row N-1 and below for vertical edges, column M-1 and beyond for
 * horizontal edges) and all padding must be zero.  The element type is
 * double for IRLSU_F64 plans and float for all other plans.
 */
#ifndef IRLSU_H
#define IRLSU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum irlsu_status {
  IRLSU_OK = 0,
  IRLSU_NOT_CONVERGED = 1,     /* warning: a PCG solve hit pcg_max */
  IRLSU_ERR_INVALID_ARG = -1,  /* null pointer, bad stride, bad parameter */
  IRLSU_ERR_SHAPE = -2,        /* N < 2 or M < 2, or sizes do not match the plan */
  IRLSU_ERR_NONFINITE = -3,    /* NaN or Inf in X or in the weights */
  IRLSU_ERR_BAD_WEIGHTS = -4,  /* a weight is <= 0 */
  IRLSU_ERR_BREAKDOWN = -5,    /* PCG breakdown: p^T A p <= 0 */
  IRLSU_ERR_HIP = -6,          /* a HIP runtime call failed */
  IRLSU_ERR_OOM = -7,          /* plan allocation failed (nothing leaked) */
  IRLSU_ERR_UNSUPPORTED = -8,  /* precision not built into this library */
  IRLSU_ERR_WORKSPACE = -9     /* workspace missing or smaller than required */
} irlsu_status;

/* Precision of a plan.  The vectors, scalars and FP64 reductions are fixed
 * by the precision alone; where the preconditioner's arithmetic runs depends
 * on the plan's form (IRLSU_PLAN_*, below):
 *   fast form (the default where it applies: power-of-two sides, or sides
 *     that are multiples of 8 whose halves have only the factors 2, 3, 5):
 *     FP32 VALU transforms
 *     (FP64 for F64 plans), the two stored intermediates in the operand
 *     type (FP16 / BF16 for the mixed plans, FP32 / FP64 otherwise);
 *   dense and folded forms (the other sides, or forced through
 *     irlsu_plan_create_ex): MFMA products with the cosine bases in the
 *     operand type, FP32 accumulation (FP64 for F64 plans). */
typedef enum irlsu_precision {
  IRLSU_F64 = 0,        /* FP64 vectors; FP64 preconditioner */
  IRLSU_F32 = 1,        /* FP32 vectors; FP32 preconditioner */
  IRLSU_MIXED_BF16 = 2, /* FP32 vectors; BF16 operands / intermediates, FP32 arithmetic */
  IRLSU_MIXED_F16 = 3   /* FP32 vectors; FP16 operands / intermediates (scaled), FP32 arithmetic */
} irlsu_precision;

typedef struct irlsu_plan irlsu_plan;

/* Solver parameters (Section 4.4 names in brackets). */
typedef struct irlsu_params {
  double eps;              /* IRLS weight floor; Omega = C / max(|r|, eps). 1e-3 */
  double pcg_rtol;         /* stop PCG when ||r|| <= pcg_rtol ||b||. 1e-8 (F64), 1e-6 otherwise */
  double l1_target;        /* > 0: stop IRLS at the first U^k with L1(U^k) <= l1_target */
  int32_t irls_iters;      /* number of IRLS iterations. 20 */
  int32_t pcg_max;         /* maximum PCG iterations per IRLS iteration. 100 */
  int32_t true_res_every;  /* recompute r = b - A u every this many PCG iterations; 0 = never. 32 */
  int32_t poll_every;      /* host reads the device convergence flag every this many PCG iterations. 4 */
  int32_t flexible;        /* CG beta: 0 = rho_new / rho (Algorithm 2), 1 = flexible
                              (z_new . (r_new - r_old) / rho), -1 = flexible for mixed plans
                              whose preconditioner runs MFMA products (dense / folded), plain
                              otherwise */
  int32_t cg_schedule;     /* IRLSU_CG_FIXED (pcg_max per solve) or IRLSU_CG_ADAPTIVE */
  int32_t cg_m0;           /* adaptive: iteration cap of the first solve, m_CG(0). 5 */
  int32_t sd_guard;        /* augmented form only (IRLSU_GUARD_*): sufficient-decrease
                              condition of Theorem 3. IRLSU_GUARD_CHECK */
  double cg_eps_tol;       /* adaptive: significance threshold of Delta. 1e-3 */
  double cg_alpha;         /* adaptive: cap growth factor. 1.7 */
  int32_t graph;           /* 1: replay each PCG iteration's launches from a captured HIP graph
                              (one graph launch instead of 5-12 kernel launches; identical
                              results); 0: launch directly. 1 */
  int32_t reserved_;
} irlsu_params;

/* CG iteration schedules (irlsu_params.cg_schedule).  The adaptive one is
 * Section 4.3: before solve k >= 1 the relative improvement Delta of the
 * IRLS model at U^k between the previous and the new weights,
 *   Delta = (S(U^k, Omega^{k-1}) - S(U^k, Omega^k)) / S(U^k, Omega^{k-1}),
 *   S(U, Omega) = sum Omega r^2 / 2 + C^2 / (2 Omega), r = DU - G,
 * keeps the cap (Delta > cg_eps_tol), stops the IRLS loop and returns U^k
 * (Delta <= cg_eps_tol right after a raise), or raises the cap to
 * ceil(cg_alpha * cap).  The missing m_CG(-1) is taken equal to m_CG(0). */
enum { IRLSU_CG_FIXED = 0, IRLSU_CG_ADAPTIVE = 1 };

/* Sufficient-decrease guard of the augmented form (irlsu_params.sd_guard).
 * Theorem 3 bounds the convergence rate of Algorithm 1 when each solve ends
 * at a point whose (prob:alt1) objective, at the weights W^k of that
 * iteration, is no larger than at the candidate gradient step
 *   x~ = x^k - grad / L,  L = 12 / tau + C_max^2 / delta,
 * (eq:candidate-gd-step).  CHECK evaluates both after every solve and takes
 * x~ when the solve did worse; CANDIDATE_ONLY takes x~ and runs no CG (the
 * variant of the remark after Theorem 3, which converges far more slowly). */
enum { IRLSU_GUARD_OFF = 0, IRLSU_GUARD_CHECK = 1, IRLSU_GUARD_CANDIDATE_ONLY = 2 };

#define IRLSU_MAX_IRLS 256

typedef struct irlsu_iter_stats {
  double L1;          /* weighted L1 objective at U^k (before solve k) */
  double H;           /* Huber objective sum C h_eps(DU - G) at U^k */
  double relres;      /* ||r|| / ||b|| of the recursive residual when solve k stopped */
  int32_t pcg_iters;  /* PCG iterations of solve k */
  int32_t status;     /* irlsu_status of solve k */
  double delta;       /* adaptive schedule: Delta before solve k (k >= 1), else 0 */
  int32_t pcg_cap;    /* iteration cap of solve k */
  int32_t guard;      /* augmented form: 0 condition not checked, 1 it held after solve k,
                         2 the candidate step of Theorem 3 replaced the solve's result */
} irlsu_iter_stats;

typedef struct irlsu_stats {
  int32_t irls_done;      /* IRLS iterations performed */
  int32_t pcg_total;      /* PCG iterations over all solves */
  int32_t target_hit;     /* 1 if l1_target was reached */
  int32_t status;         /* overall status */
  double L1_final;        /* L1 of the returned U */
  double H_final;         /* Huber objective of the returned U */
  int32_t schedule_stop;  /* 1 if the adaptive schedule ended the IRLS loop */
  int32_t reserved_;
  irlsu_iter_stats iter[IRLSU_MAX_IRLS];
} irlsu_stats;

typedef struct irlsu_plan_desc {
  int64_t N, M;           /* image rows, columns */
  int64_t Np, ld;         /* padded rows, padded row stride (elements) */
  int32_t precision;      /* irlsu_precision */
  int32_t elem_bytes;     /* 8 for F64 plans, 4 otherwise */
  size_t workspace_bytes; /* workspace needed by irlsu_unwrap and the step functions */
  size_t plan_bytes;      /* device memory owned by the plan (basis, eigenvalues) */
  int32_t folded;         /* 1: preconditioner in the folded (even/odd) form */
  int32_t form;           /* IRLSU_PLAN_DENSE, _FOLDED or _FAST: the form in use */
} irlsu_plan_desc;

/* Form of the preconditioner products (irlsu_plan_create_ex). */
enum {
  IRLSU_PLAN_AUTO = 0,   /* fast where the fast form applies (below);
                            else folded when N, M are even and N M >= 2^20;
                            else dense */
  IRLSU_PLAN_DENSE = 1,  /* four dense MFMA products (Section 3.3 as written) */
  IRLSU_PLAN_FOLDED = 2, /* reflection symmetry of the DCT-II basis: each product
                            splits into even / odd halves, half the MFMA work;
                            N and M must be even (else ERR_SHAPE) */
  IRLSU_PLAN_FAST = 3    /* the same products by fast cosine transforms
                            (half-length FFTs in LDS, FP32 arithmetic for FP32
                            and mixed plans, FP64 for FP64 plans); N and M
                            both powers of two in [128, 16384], or each a
                            multiple of 8 whose half is at most 8192 and has
                            no prime factor above 5 (4000, 6000, 16000, ...);
                            else ERR_SHAPE */
};

/* Testing hook for the ERR_OOM path (for callers that test their own error
 * handling): with nth >= 0, the nth (from 0) device or pinned host
 * allocation made by the following plan and batch creations fails as if
 * the device were out of memory, after which the hook disarms itself; a
 * negative nth disarms it.  Process-wide and not thread-safe. */
void irlsu_test_fail_alloc(int32_t nth);

/* Human-readable name of a status code (static storage). */
const char* irlsu_status_string(irlsu_status st);

/* Fill *p with the defaults for precision prec. */
irlsu_status irlsu_params_default(irlsu_params* p, irlsu_precision prec);

/* Create a plan for N x M images (Section 3.3, eq:eigendecompositions: what
 * the preconditioner needs is computed once and reused by every PCG
 * iteration).  The form is chosen as IRLSU_PLAN_AUTO describes; on the
 * current HIP device the plan allocates and fills
 *   fast form: the FFT twiddle tables of each side (about 3n/2 complex
 *     values per side -- the stage twiddles for power-of-two plans, the
 *     n/2-th roots of unity otherwise -- and n/4 + 1 records of the
 *     column pass's pair twiddles and eigenvalues, shared when N = M) and
 *     the Laplacian eigenvalues
 *     2 - 2 cos(pi k / n) in FP64;
 *   dense form: the orthonormal DCT-II bases P_N, P_M and their transposes
 *     in the operand type, and the eigenvalues;
 *   folded form: the even / odd half bases and the eigenvalues.
 * Synchronises the stream before returning.
 * Sizes: 2 <= N, M <= 32768.
 * Errors: ERR_INVALID_ARG (out null), ERR_SHAPE, ERR_UNSUPPORTED, ERR_OOM,
 * ERR_HIP.  On error *out is NULL and nothing is leaked. */
irlsu_status irlsu_plan_create(irlsu_plan** out, int64_t N, int64_t M,
                               irlsu_precision prec, void* stream);

/* As irlsu_plan_create, choosing the form of the preconditioner
 * (IRLSU_PLAN_AUTO / _DENSE / _FOLDED / _FAST); every form computes the
 * same map. */
irlsu_status irlsu_plan_create_ex(irlsu_plan** out, int64_t N, int64_t M,
                                  irlsu_precision prec, int32_t form, void* stream);

/* Release a plan and its device memory.  NULL is accepted. */
irlsu_status irlsu_plan_destroy(irlsu_plan* plan);

/* Describe a plan (host struct). */
irlsu_status irlsu_plan_info(const irlsu_plan* plan, irlsu_plan_desc* out);

/* Workspace bytes needed by irlsu_unwrap and the step functions (0 on NULL). */
size_t irlsu_workspace_bytes(const irlsu_plan* plan);

/* Unwrap one image (the whole hot path: setup, IRLS weight updates, PCG with
 * the DCT preconditioner, mean removal).  Section 2 problem, Algorithm 1.
 *
 *   X       device, N x M wrapped phase, row stride ldx >= M elements.
 *   w       device or NULL: N x M per-pixel weights > 0 (stride ldx); edge
 *           weight = min of its two pixel weights.
 *   Cv, Ch  device or NULL (both or neither; override w): per-edge weights
 *           > 0, Cv (N-1) x M with stride ldcv >= M, Ch N x (M-1) with
 *           stride ldch >= M-1.  With no weights, C = 1.
 *   U0      device or NULL: N x M warm start (stride ldu), e.g. to resume.
 *   params  host or NULL (defaults for the plan's precision).
 *   U       device out: N x M mean-zero unwrapped phase (stride ldu >= M).
 *           May alias U0.
 *   workspace, workspace_bytes: device scratch owned by the caller, at least
 *           irlsu_workspace_bytes(plan); contents are overwritten.
 *   stats   host or NULL.
 *
 * Element type of X, w, Cv, Ch, U0, U: double for F64 plans, float otherwise.
 * The call synchronises the stream once after setup (input validation) and
 * whenever it reads the device convergence flag (every poll_every PCG
 * iterations) or the objectives (every IRLS iteration when stats or
 * l1_target are given).  Returns OK, NOT_CONVERGED (a solve hit pcg_max;
 * U is still valid), or an error: ERR_INVALID_ARG, ERR_SHAPE,
 * ERR_NONFINITE, ERR_BAD_WEIGHTS, ERR_BREAKDOWN, ERR_WORKSPACE, ERR_HIP. */
irlsu_status irlsu_unwrap(irlsu_plan* plan,
                          const void* X, int64_t ldx,
                          const void* w,
                          const void* Cv, int64_t ldcv,
                          const void* Ch, int64_t ldch,
                          const void* U0,
                          const irlsu_params* params,
                          void* U, int64_t ldu,
                          void* workspace, size_t workspace_bytes,
                          irlsu_stats* stats, void* stream);

/* ---- Batched uneven tiles ---------------------------------------------- */

typedef struct irlsu_batch irlsu_batch;

/* One independent problem of a batch (each tile is its own Section 2
 * problem with its own mean-zero constraint; tiles are not coupled).  Same
 * argument meaning and layout as irlsu_unwrap, element type float. */
typedef struct irlsu_tile {
  const void* X; int64_t ldx;
  const void* w;
  const void* Cv; int64_t ldcv;
  const void* Ch; int64_t ldch;
  void* U; int64_t ldu;
} irlsu_tile;

/* Create a batch for ntiles tiles of shapes[2t] x shapes[2t+1] (host array).
 * Builds one DCT-II basis per distinct side length (Section 3.3 precompute)
 * in the mixed precisions only (IRLSU_MIXED_BF16 or IRLSU_MIXED_F16; other
 * precisions return ERR_UNSUPPORTED).  Tiles are padded to multiples of 256.
 * Errors as irlsu_plan_create; ERR_SHAPE also when the batch is too large
 * for the partial-sum table. */
irlsu_status irlsu_batch_create(irlsu_batch** out, const int64_t* shapes, int32_t ntiles,
                                irlsu_precision prec, void* stream);
irlsu_status irlsu_batch_destroy(irlsu_batch* batch);
size_t irlsu_batch_workspace_bytes(const irlsu_batch* batch);

/* Unwrap all tiles of a batch.  Every PCG phase (stencil, update,
 * preconditioner products) is one grouped launch over all tiles, with
 * per-tile scalars and convergence flags; converged tiles drop out.
 * tiles: host array of ntiles descriptors; stats: host array of ntiles or
 * NULL.  Returns the worst per-tile status. */
irlsu_status irlsu_unwrap_batched(irlsu_batch* batch, const irlsu_tile* tiles,
                                  const irlsu_params* params, void* workspace,
                                  size_t workspace_bytes, irlsu_stats* stats, void* stream);

/* Adjoint of the converged system (frozen weights).  For a loss L(U) with
 * gU = dL/dU (device, N x M, stride ldg), differentiates the map
 * (C, X) -> U = argmin over mean-zero U of sum C omega (DU - G(X))^2 with
 * omega = 1 / max(|DU* - G|, eps) frozen at the U* that the last
 * irlsu_unwrap on this plan and workspace returned (the fixed point of
 * Algorithm 1).  One extra PCG solve D^T Omega D lambda = gU - mean(gU) with
 * the forward kernels, then per edge gC = -omega (D lambda) (DU* - G) and
 * gX = D^T (Omega D lambda).
 *   gCv (N-1) x M (stride ldgcv), gCh N x (M-1) (stride ldgch): device out.
 *   gX  N x M (stride ldgx): device out, nullable.
 *   workspace: the one passed to the preceding irlsu_unwrap, unmodified since.
 *   params: solver parameters of the adjoint solve (NULL: defaults).
 * Returns OK, NOT_CONVERGED or an error as irlsu_unwrap; stats (nullable)
 * gets the solve's iteration count and relative residual in iter[0]. */
irlsu_status irlsu_adjoint(irlsu_plan* plan, const void* gU, int64_t ldg,
                           const irlsu_params* params,
                           void* gCv, int64_t ldgcv, void* gCh, int64_t ldgch,
                           void* gX, int64_t ldgx,
                           void* workspace, size_t workspace_bytes,
                           irlsu_stats* stats, void* stream);

/* Full implicit derivative of the Huber minimiser.  The same arguments as
 * irlsu_adjoint, for the map (C, X) -> U* = argmin over mean-zero U of
 * sum C h_eps(DU - G(X)) (the problem whose minimiser the IRLS fixed point
 * is, Section 3 with the reduced weights), differentiated through its
 * stationarity condition D^T (C h_eps'(DU* - G)) = 0: with r = DU* - G and
 * the Hessian weights kappa = C / eps on the quadratic zone |r| < eps (0 off
 * it), lambda solves D^T diag(kappa) D lambda = gU (projected), then
 *   gC = -h_eps'(r) (D lambda),  gX = D^T (kappa D lambda),
 * h_eps'(r) = r / eps on the zone, sign(r) off it.  Pixels with no
 * quadratic-zone edge are left out (the minimiser is not unique there): gU
 * is taken as zero on them and lambda = 0 there, with lambda of mean zero
 * over the others.  The remaining pixels must be connected through
 * quadratic-zone edges; otherwise the solve cannot converge and
 * NOT_CONVERGED is returned.  The workspace's weight arrays are overwritten
 * (by kappa). */
irlsu_status irlsu_adjoint_implicit(irlsu_plan* plan, const void* gU, int64_t ldg,
                                    const irlsu_params* params,
                                    void* gCv, int64_t ldgcv, void* gCh, int64_t ldgch,
                                    void* gX, int64_t ldgx,
                                    void* workspace, size_t workspace_bytes,
                                    irlsu_stats* stats, void* stream);

/* ---- Launch-shape autotuner ------------------------------------------- */

/* Launch shapes of a plan.  0 everywhere: the library's default rules. */
typedef struct irlsu_tune {
  int32_t stencil_rows;   /* rows of the image per operator workgroup (its band height) */
  int32_t update_blocks;  /* workgroups of the CG update (at most the operator's) */
  int32_t small_tiles;    /* 16-bit MFMA products: 1 = 128 x 128 tiles, 0 = 256 x 256 where
                             they divide the padded sides */
  int32_t from_cache;     /* out: 1 if the shapes came from the cache file */
  double stencil_us;      /* out: measured time of the chosen shapes, microseconds */
  double update_us;
  double precond_us;      /* 16-bit MFMA forms only, else 0 */
} irlsu_tune;

/* Choose the launch shapes of a plan by measurement: every candidate band
 * height of the operator (8 .. 256 rows), update block count (64 .. 4096)
 * and, for 16-bit MFMA forms, product tile, timed with HIP events on
 * `stream` on the plan's workspace (its contents are overwritten); the
 * fastest of each is applied to the plan.  With cache_path non-NULL the
 * choice is first looked up in that JSON file, keyed by N, M, precision,
 * form and the GPU's architecture name, and a new measurement is stored
 * there (the file is rewritten whole).  Results of the solves do not
 * depend on the shapes beyond the summation order of the FP64 partial
 * sums.  Synchronises the stream.  out (host, nullable) gets the choice.
 * Errors: ERR_INVALID_ARG (null plan, or the cache file cannot be written),
 * ERR_WORKSPACE, ERR_HIP. */
irlsu_status irlsu_plan_autotune(irlsu_plan* plan, const char* cache_path, irlsu_tune* out,
                                 void* workspace, size_t workspace_bytes, void* stream);

/* Force a plan's launch shapes (NULL: back to the default rules).  Errors:
 * ERR_INVALID_ARG (null plan, negative fields, small_tiles not 0 or 1). */
irlsu_status irlsu_plan_set_tune(irlsu_plan* plan, const irlsu_tune* tune);

/* The plan's current launch shapes (0: default rule).  Errors:
 * ERR_INVALID_ARG. */
irlsu_status irlsu_plan_get_tune(const irlsu_plan* plan, irlsu_tune* out);

/* The batch's operator band heights, one per distinct tile shape, chosen by
 * measurement of each tile's operator alone (cached like
 * irlsu_plan_autotune's, as kind "batch_tile"); the grouped launches then
 * use them.  The workspace's contents are overwritten.  Errors:
 * ERR_INVALID_ARG, ERR_WORKSPACE, ERR_HIP. */
irlsu_status irlsu_batch_autotune(irlsu_batch* batch, const char* cache_path, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* ---- Step-level entry points (internal layout, see top of file) -------- */

/* Setup (Section 2): Gv, Gh = wrapped differences W(d) = d - 2 pi
 * floor((d + pi) / 2 pi) of X computed in FP64, stored in the plan's
 * element type; CvI, ChI = per-edge weights by the irlsu_unwrap rules.  All
 * four outputs are device, internal layout.  Input arguments as in
 * irlsu_unwrap.  Also validates the inputs: *flags (device int32) gets bit 0
 * for a non-finite value and bit 1 for a weight <= 0 (caller zeroes it). */
irlsu_status irlsu_setup(const irlsu_plan* plan,
                         const void* X, int64_t ldx, const void* w,
                         const void* Cv, int64_t ldcv,
                         const void* Ch, int64_t ldch,
                         void* Gv, void* Gh, void* CvI, void* ChI,
                         int32_t* flags, void* stream);

/* IRLS weight step (closed-form weights, Section 3.1): with r = DU - G,
 * Ov/Oh = C / max(|r|, eps), b = D^T (Omega G), and objectives[0..2] =
 * {sum C |r|, sum C h_eps(r), ||b||^2} accumulated in FP64 (device doubles).
 * All images device, internal layout.  workspace as for irlsu_unwrap. */
irlsu_status irlsu_weights(const irlsu_plan* plan, double eps,
                           const void* U, const void* Gv, const void* Gh,
                           const void* CvI, const void* ChI,
                           void* Ov, void* Oh, void* b, double* objectives,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Weighted 5-point operator q = D^T Omega D p (the U block of the system of
 * Proposition 1 after slack elimination; Appendix A gives S^T S and T T^T).
 * p, q, Ov, Oh device, internal layout; q must not alias p.  pq (device
 * double, nullable) receives sum p q accumulated in FP64. */
irlsu_status irlsu_operator(const irlsu_plan* plan, const void* Ov, const void* Oh,
                            const void* p, void* q, double* pq,
                            void* workspace, size_t workspace_bytes, void* stream);

/* irlsu_operator for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernel and the same result, bit for bit, with no workspace.  The
 * per-block partial sums of p . q live in a scratch array of the library
 * (96 KiB of device memory on each GPU it runs on, held until the process
 * ends); the call allocates nothing, neither device nor host memory.
 * Arguments and layout as irlsu_operator; the plan must belong to the
 * current device.  Limit: images whose operator launch has at most 4096
 * blocks -- ceil(ld / 1024) * ceil(Np / 64) <= 4096, e.g. up to
 * 16384 x 16384 -- larger plans return ERR_SHAPE.  Every call on one GPU
 * shares that GPU's scratch: calls that overlap in time on one GPU (on
 * different streams, or from several threads) race and must be serialised
 * by the caller.  Errors: ERR_INVALID_ARG (null pointer, p == q, plan of
 * another device), ERR_SHAPE, ERR_HIP. */
irlsu_status irlsu_operator_noalloc(const irlsu_plan* plan, const void* Ov, const void* Oh,
                                    const void* p, void* q, double* pq, void* stream);

/* Preconditioner z = L^+ r (Section 3.3, Appendix B): orthonormal DCT-II of
 * both axes, division by lambda_k + mu_l, mode (0,0) set to zero, DCT-III
 * back.  How the transforms run is the plan's form: fast cosine transforms
 * on the VALU in FP32 (FP64 for F64 plans) with the intermediates stored in
 * the operand type (fast form), or products with the cosine bases on MFMA
 * with FP32 accumulation (FP64 for F64 plans; dense and folded forms).
 * r, z device, internal layout, may not alias.  rz (device double,
 * nullable) receives sum r z in FP64. */
irlsu_status irlsu_precond(const irlsu_plan* plan, const void* r, void* z, double* rz,
                           void* workspace, size_t workspace_bytes, void* stream);

/* PCG solve (Algorithm 2) of D^T Omega D x = b for given weights: the
 * solve inside each IRLS iteration, on its own.  The preconditioner is the
 * plan's L^+ (Section 3.3), the stopping rule ||r|| <= pcg_rtol ||b|| on the
 * recursive residual, at most pcg_max iterations, the true residual
 * recomputed every true_res_every iterations (params as irlsu_unwrap; NULL:
 * defaults).  b is projected on the range of the operator (its mean over
 * the N x M pixels removed), since D^T Omega D annihilates constants.
 *   Ov, Oh, b  device, internal layout, plan element type (copied into the
 *              workspace; weights of missing edges and padding zero).
 *   x          device, Np x ld doubles (FP64 for every precision: the
 *              iterate is FP64, each solve accumulates its correction in
 *              the vector type and adds it once): warm start in, solution
 *              out (not mean-adjusted); padding must be zero.
 *   iters, relres  host, nullable: iterations performed and the final
 *              ||r|| / ||b||.
 * Synchronises the stream (polls the device convergence flag).  Returns
 * OK, NOT_CONVERGED (pcg_max reached), ERR_BREAKDOWN (p^T A p <= 0 or
 * rho < 0, e.g. for weights that are not positive), ERR_INVALID_ARG,
 * ERR_WORKSPACE, ERR_HIP. */
irlsu_status irlsu_pcg(irlsu_plan* plan, const void* Ov, const void* Oh, const void* b,
                       double* x, const irlsu_params* params, int32_t* iters, double* relres,
                       void* workspace, size_t workspace_bytes, void* stream);

/* The paper's augmented form (Algorithm 1 in (U, V^v, V^h) with tau and
 * delta): closed-form weights W = sqrt(C^2 V^2 + delta^2), then Algorithm 2
 * on the symmetric system of Proposition 1 preconditioned by the block
 * diagonal of Section 3.3 (tau L^+ on U, (C^2/W + 1/tau)^-1 on V), warm
 * started, then mean removal of U.  U^0 = 0, V^0 = D U^0 - G.  Inputs and
 * output as irlsu_unwrap (no warm start); params as irlsu_unwrap (eps and
 * the schedule fields are not used; l1_target stops at the first U^k with
 * L1 <= l1_target; sd_guard selects the Theorem 3 guard, IRLSU_GUARD_*).
 * stats: iter[k].L1 = L1(U^k), iter[k].H = F_delta(U^k, V^k) (the
 * objective of the smoothed problem), iter[k].guard the guard's outcome of
 * solve k.  The workspace (irlsu_augmented_workspace_bytes) is larger than
 * irlsu_unwrap's (three more vectors of each block hold the candidate).
 * Errors: ERR_INVALID_ARG (tau or delta <= 0, sd_guard outside 0..2,
 * strides, nulls),
 * ERR_WORKSPACE, ERR_NONFINITE, ERR_BAD_WEIGHTS, ERR_BREAKDOWN, ERR_HIP;
 * NOT_CONVERGED as irlsu_unwrap. */
size_t irlsu_augmented_workspace_bytes(const irlsu_plan* plan);
irlsu_status irlsu_unwrap_augmented(irlsu_plan* plan, const void* X, int64_t ldx,
                                    const void* w, const void* Cv, int64_t ldcv,
                                    const void* Ch, int64_t ldch, const irlsu_params* params,
                                    double tau, double delta, void* U, int64_t ldu,
                                    void* workspace, size_t workspace_bytes,
                                    irlsu_stats* stats, void* stream);

/* Rounded output ("rounded IRLS" of the experiments, Section 4): writes
 * out = X + 2 pi rint((U + c - X) / 2 pi) with c = arg sum exp(i (X - U)),
 * i.e. U (defined up to a constant) aligned with X modulo 2 pi and rounded
 * to the nearest image that is 2 pi-congruent to X.  X, U and out are
 * N x M device arrays of the plan's element type (row strides ldx, ldu,
 * ldo >= M, elements); out may alias U.  Uses the workspace's reduction
 * slots.  Errors: ERR_INVALID_ARG, ERR_WORKSPACE, ERR_HIP. */
irlsu_status irlsu_round_congruent(const irlsu_plan* plan, const void* X, int64_t ldx,
                                   const void* U, int64_t ldu, void* out, int64_t ldo,
                                   void* workspace, size_t workspace_bytes, void* stream);

/* Kinds of launch reported by irlsu_precond_timed and irlsu_profile_result. */
#define IRLSU_MAX_LAUNCHES 32
enum {
  IRLSU_LK_PRODUCT = 0,    /* MFMA product with the cosine basis (dense / folded) */
  IRLSU_LK_ROWS_DCT2 = 1,  /* fast form: DCT-II along rows */
  IRLSU_LK_TRANSPOSE = 2,  /* fast form: transpose */
  IRLSU_LK_COLS = 3,       /* fast form: DCT-II, division, DCT-III along columns */
  IRLSU_LK_ROWS_DCT3 = 4,  /* fast form: DCT-III along rows with z.r, z.q, sum z */
  IRLSU_LK_BUTTERFLY = 5,  /* folded form: sum / difference pass */
  IRLSU_LK_DOTS = 6,       /* z.r, z.q, sum z pass (with the recombination when folded) */
  IRLSU_LK_PROLOGUE = 7,   /* convergence test and input scale */
  IRLSU_LK_PARTIALS = 8,   /* fold of per-block partial sums */
  IRLSU_LK_STENCIL = 9,    /* p = z + beta p, q = D^T Omega D p, p.q (PCG loop form) */
  IRLSU_LK_AXPY = 10,      /* alpha, d += alpha p, r -= alpha q, ||r||^2 */
  IRLSU_LK_RESIDUAL = 11,  /* true-residual refresh r = b - A (u + d) */
  IRLSU_LK_UPDATE_DCT2 = 12, /* fast form: r -= alpha q fused with the DCT-II along
                                rows of the new r (d += alpha p then rides on the
                                DCT-III along rows, which reads p anyway) */
  IRLSU_LK_ALPHA = 13      /* alpha = rho / p.q and the FP16 input scale */
};

/* Timing of the preconditioner of Section 3.3 (the products named there as
 * the main cost): reps applications of irlsu_precond's map, with a HIP event
 * recorded on `stream` before the first launch and after every launch.
 * Writes, for each of the *n_launches launches of one application (at most
 * IRLSU_MAX_LAUNCHES), its mean duration over the reps in ms_launch[i] and
 * its IRLSU_LK_* kind in kind[i]; z receives the last application.
 * Synchronises the stream.  Errors as irlsu_precond; ERR_INVALID_ARG also
 * for reps < 1 or a null output pointer; ERR_HIP when events cannot be
 * created. */
irlsu_status irlsu_precond_timed(const irlsu_plan* plan, const void* r, void* z,
                                 void* workspace, size_t workspace_bytes, int32_t reps,
                                 double* ms_launch, int32_t* kind, int32_t* n_launches,
                                 void* stream);

/* Measurement aid: the HBM ceilings that the kernels' bandwidth is reported
 * against.  Streams `bytes` (a multiple of 16) with the library's own
 * streaming kernel: IRLSU_PROBE_COPY reads a and writes d, IRLSU_PROBE_READ
 * reads a only (d may be NULL), IRLSU_PROBE_3R1W reads a, b, c and writes
 * d (the operator's mix).  grid blocks of 256 threads, 16-byte
 * non-temporal accesses; one warm-up launch, then reps launches timed with
 * HIP events on `stream`; *ms gets the mean per launch.  All buffers are
 * device memory of at least `bytes`.  Synchronises the stream.  Errors:
 * ERR_INVALID_ARG, ERR_HIP. */
enum { IRLSU_PROBE_COPY = 0, IRLSU_PROBE_READ = 1, IRLSU_PROBE_3R1W = 2 };
irlsu_status irlsu_stream_probe(int32_t kind, const void* a, const void* b, const void* c, void* d,
                                size_t bytes, int32_t grid, int32_t reps, double* ms,
                                void* stream);

/* Timing aid for one iteration of Algorithm 2 inside irlsu_unwrap: arms the
 * plan so that the next irlsu_unwrap records a HIP event on its stream after
 * every launch of PCG iteration pcg_l of IRLS iteration irls_k (operator,
 * axpy, true-residual refresh if due, preconditioner passes).  A negative
 * index disarms.  The recording stays with the plan until the next arm.
 * Errors: ERR_INVALID_ARG (null plan), ERR_OOM, ERR_HIP. */
irlsu_status irlsu_profile_arm(irlsu_plan* plan, int32_t irls_k, int32_t pcg_l);

/* Durations (ms) and IRLSU_LK_* kinds of the launches recorded for the armed
 * iteration, in launch order (at most IRLSU_MAX_LAUNCHES); *n_launches = 0
 * when the iteration was not reached.  Waits for the recorded events.
 * Errors: ERR_INVALID_ARG (null argument), ERR_HIP. */
irlsu_status irlsu_profile_result(irlsu_plan* plan, double* ms_launch, int32_t* kind,
                                  int32_t* n_launches);

#ifdef __cplusplus
}
#endif

#endif /* IRLSU_H */
