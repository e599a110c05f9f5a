// Kernel argument blocks and launchers of the irlsu library.
#pragma once

#include "common.hpp"

namespace irlsu {

template <class T>
struct SetupArgs {
  const T* X; int64_t ldx;
  const T* w;                       // nullable per-pixel weights (stride ldx)
  const T* Cv; int64_t ldcv;        // nullable per-edge weights
  const T* Ch; int64_t ldch;
  const T* U0; int64_t ldu0;        // nullable warm start
  int64_t N, M, Np, ld;
  T* Gv; T* Gh; T* Cv_out; T* Ch_out;
  double* U;                        // nullable: internal U to initialise
  int32_t* flags;                   // input-validation bits
};

template <class T>
struct WeightsArgs {
  const double* U;
  const T* Gv; const T* Gh; const T* Cv; const T* Ch;
  T* Ov; T* Oh; T* b;
  double eps;
  int64_t Np, ld;
  DevState st;
  int want_model = 0;   // also sum the IRLS model at U with the previous and new weights
};

template <class T>
struct AxpyArgs {
  double* u; T* r; const T* p; const T* q;
  T* d = nullptr;     // non-null: the solve's correction d += alpha p (vector
                      // type); u is then left alone until the solve ends
  int64_t n;          // Np * ld, a multiple of 4
  int nparts_pq;      // number of p.q partials written by the stencil
  int nparts_out = 0; // partials the consumers of ||r||^2 and sum r read (the
                      // stencil's count); slots beyond the grid are zeroed
  int iter;
  DevState st;
};

// Weighted 5-point stencil modes.
enum StencilMode : int {
  ST_FUSED = 0,   // p = (z - zc) + beta p_old;  q = A p;  partial p.q
  ST_APPLY = 1,   // q = A p;  partial p.q
  ST_RESID = 2,   // r = b - A u (u in FP64);  partial ||r||^2, sum r
};

template <class T>
struct StencilArgs {
  const T* Ov; const T* Oh;
  const T* z;          // FUSED: preconditioned residual
  const T* p_in;       // FUSED: previous direction; APPLY: p
  T* p_out;            // FUSED: new direction (must not alias p_in)
  T* q;                // FUSED / APPLY output
  const double* u;     // RESID input
  const T* d = nullptr;  // RESID: correction of the current solve (u + d)
  const T* b;          // RESID input
  T* r;                // RESID output
  int64_t N, M, Np, ld;
  int iter;            // FUSED: PCG iteration l (l == 0 -> beta = 0)
  int flexible;        // FUSED: flexible beta
  int nparts_prec;     // FUSED: partials of the preconditioner epilogue
  int nparts_res;      // FUSED: partials of sum r (axpy or residual kernel)
  int check_done;      // skip when the PCG done flag is set
  int want_qq = 0;     // APPLY: also the partial ||q||^2 (slot PR_AUX)
  int nparts_out = 0;  // RESID: partial count the consumers read (zero padded)
  int rows = 0;        // band height of a block (0: the default rule of stencil_grid)
  DevState st;
};

// ---- batched tiles ------------------------------------------------------
// Device-resident description of one tile of a batch: its sizes, its
// vectors in the internal layout, its scalars and partial range, its grids
// and its preconditioner (basis tables of its side lengths).
template <class T>
struct BatchTile {
  int64_t N, M, Np, ld;
  double* U;
  T* r; T* z; T* p0; T* p1; T* q; T* b; T* Ov; T* Oh;
  DevState st;
  int32_t st_gx, st_rows, st_nblk;   // stencil grid: column blocks, rows per band, blocks
  int32_t g4_nparts;                 // partials of the last preconditioner product
  int32_t flexible_q;                // pass q to the preconditioner epilogue
  int32_t fast;                      // preconditioner in the fast form (its own launches)
  void* T1; void* T2; void* T3;
  const void* PN; const void* PNt; const void* PM; const void* PMt;
  const double* eigN; const double* eigM;
};

// Index t with start[t] <= b < start[t + 1] (start has ntiles + 1 entries).
__device__ __forceinline__ int find_tile(const int32_t* start, int ntiles, int b) {
  int lo = 0, hi = ntiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T>
struct StencilArgs;

template <class T> void launch_setup(const SetupArgs<T>& a, hipStream_t s);
template <class T> int launch_weights(const WeightsArgs<T>& a, hipStream_t s);
void launch_finalize_weights(DevState st, int nparts, double* out, double tol2, hipStream_t s,
                             int want_model = 0);
template <class T> int launch_axpy(const AxpyArgs<T>& a, hipStream_t s, int nblocks);
int axpy_blocks(int stencil_blocks);
// out = X + 2 pi rint((U + c - X) / 2 pi), c = arg sum exp(i (X - U))
template <class T>
void launch_congruent(const T* X, int64_t ldx, const T* U, int64_t ldu, T* out, int64_t ldo,
                      int64_t N, int64_t M, DevState st, hipStream_t s);
// u += d (FP64) over n elements: the end of a solve; with clear, also d = 0
// (a true-residual refresh moves the correction so far into u)
template <class T>
void launch_commit(double* u, T* d, int64_t n, hipStream_t s, bool clear = false);
void launch_mean_removal(double* u, int64_t N, int64_t M, int64_t ld, DevState st, hipStream_t s);
template <class T>
void launch_copy_out(const double* u, int64_t ld, T* out, int64_t ldo, int64_t N, int64_t M,
                     hipStream_t s);
void launch_finalize_rr(DevState st, int nparts, hipStream_t s);
void launch_reduce_to(DevState st, int slot, int nparts, double* out, hipStream_t s);
int elementwise_blocks(int64_t n);
dim3 weights_grid(int64_t Np, int64_t ld, int* rows_out);
template <class T> int launch_sumsq(const T* x, int64_t n, DevState st, hipStream_t s);

template <class T> int launch_stencil(int mode, const StencilArgs<T>& a, hipStream_t s);

// streaming bandwidth probe (kind 0 copy, 1 read, 2 three reads + one write)
int launch_stream_probe(int kind, const void* a, const void* b, const void* c, void* d,
                        size_t bytes, int grid, int reps, float* ms, hipStream_t s);

template <class T>
__device__ __forceinline__ StencilArgs<T> batch_stencil_args(const BatchTile<T>& bt, int mode,
                                                            int iter, int flexible, int check_done) {
  StencilArgs<T> a;
  a.Ov = bt.Ov;
  a.Oh = bt.Oh;
  a.z = bt.z;
  a.p_in = (iter & 1) ? bt.p0 : bt.p1;
  a.p_out = (iter & 1) ? bt.p1 : bt.p0;
  a.q = bt.q;
  a.u = bt.U;
  a.b = bt.b;
  a.r = bt.r;
  a.N = bt.N;
  a.M = bt.M;
  a.Np = bt.Np;
  a.ld = bt.ld;
  a.iter = iter;
  a.flexible = flexible;
  a.nparts_prec = bt.g4_nparts;
  a.nparts_res = bt.st_nblk;
  a.check_done = check_done;
  a.st = bt.st;
  (void)mode;
  return a;
}
template <class T>
void launch_stencil_batched(int mode, const BatchTile<T>* tiles, const int32_t* start, int ntiles,
                            int total_blocks, int iter, int flexible, int check_done,
                            hipStream_t s);
template <class T>
void launch_axpy_batched(const BatchTile<T>* tiles, const int32_t* start, int ntiles,
                         int total_blocks, int iter, hipStream_t s);
// Grid of the stencil (and of the axpy, which must write as many partials).
dim3 stencil_grid(int64_t Np, int64_t ld, int* rows_out, int force_rows = 0);

// ---- adjoint (frozen-weight) -------------------------------------------
template <class T>
struct AdjEdgeArgs {
  const double* U; const double* lam;
  const T* Gv; const T* Gh; const T* Cv; const T* Ch;   // internal layout
  double eps;
  int64_t N, M, ld;
  T* gCv; int64_t ldgcv;    // (N-1) x M, caller layout
  T* gCh; int64_t ldgch;    // N x (M-1)
  T* gX; int64_t ldgx;      // N x M, nullable
  // full implicit derivative of the Huber minimiser: the Hessian weights
  // (kappa, internal layout; pixels with no kappa > 0 edge are left out) and
  // the mean of lambda over the other pixels (device scalar)
  const T* Kv = nullptr; const T* Kh = nullptr;
  const double* lam_mean = nullptr;
};
template <class T>
void launch_adjoint_rhs(const T* g, int64_t ldg, int64_t N, int64_t M, int64_t Np, int64_t ld,
                        T* b, DevState st, double tol2, hipStream_t s);
template <class T> void launch_adjoint_edges(const AdjEdgeArgs<T>& a, hipStream_t s);
// kappa = C / eps where |DU - G| < eps, else 0, into Kv, Kh (internal layout)
template <class T>
void launch_adjoint_hessian(const double* U, const T* Gv, const T* Gh, const T* Cv, const T* Ch,
                            double eps, int64_t N, int64_t M, int64_t Np, int64_t ld, T* Kv, T* Kh,
                            hipStream_t s);
// b = gU - mean(gU) over the pixels with a kappa > 0 edge, 0 on the others
template <class T>
void launch_adjoint_rhs_implicit(const T* g, int64_t ldg, int64_t N, int64_t M, int64_t Np,
                                 int64_t ld, const T* Kv, const T* Kh, T* b, DevState st,
                                 double tol2, hipStream_t s);
// mean of lambda over the pixels with a kappa > 0 edge into sc[SC_MEAN]
template <class T>
void launch_adjoint_lam_mean(const double* lam, int64_t N, int64_t M, int64_t ld, const T* Kv,
                             const T* Kh, DevState st, hipStream_t s);

// ---- DCT preconditioner (dense cosine-basis products on MFMA) ----------
enum OperandKind : int { OK_F64 = 0, OK_F32 = 1, OK_BF16 = 2, OK_F16 = 3 };

// Optional per-launch timing of one preconditioner application: an event
// is recorded before the first launch and after every launch, each launch
// tagged with its kind (IRLSU_LK_* of the public header).
struct LaunchLog {
  static constexpr int kMax = IRLSU_MAX_LAUNCHES;
  hipEvent_t ev[kMax + 1];
  int cls[kMax];
  int n = 0;
};
// Opens the log (first event) unless launches are already recorded in it,
// so a caller can time a sequence that contains a preconditioner.
inline void log_start(LaunchLog* L, hipStream_t s) {
  if (L && L->n == 0) (void)hipEventRecord(L->ev[0], s);
}
inline void log_mark(LaunchLog* L, int kind, hipStream_t s) {
  if (L && L->n < LaunchLog::kMax) {
    L->cls[L->n] = kind;
    (void)hipEventRecord(L->ev[++L->n], s);
  }
}

struct PrecondArgs {
  int kind;                 // OperandKind
  int64_t N, M, Np, Mp;     // Mp == ld
  const void* PN;  const void* PNt;   // Np x Np basis and its transpose (operand type)
  const void* PM;  const void* PMt;   // Mp x Mp
  const void* eigN; const void* eigM; // inverse-eigenvalue tables (see dct.hip)
  void* T1; void* T2; void* T3;       // intermediates (operand type), Np * Mp each
  const void* r;            // residual (T)
  void* z;                  // output (T)
  const void* q;            // nullable: previous A p for the flexible beta (T)
  int check_conv;           // first product checks ||r|| <= tol ||b|| and stops
  int nparts_rr;            // partials of ||r||^2 for the convergence check
  DevState st;
  // folded form (even N and M): half-size bases, even-first eigenvalue
  // tables (length 2 hNp / 2 hMp), two ping-pong operand buffers of
  // 2 hNp x 2 hMp elements and an FP32/FP64 buffer of Np x 2 hMp.
  int folded = 0;
  int64_t hNp = 0, hMp = 0;
  const void *PeN = nullptr, *PeNt = nullptr, *PoN = nullptr, *PoNt = nullptr;
  const void *PeM = nullptr, *PeMt = nullptr, *PoM = nullptr, *PoMt = nullptr;
  const void *eigNf = nullptr, *eigMf = nullptr;
  void* ZEO = nullptr;
  // fast form (power-of-two sides): twiddle tables per side; eigN / eigM
  // are then unpadded natural-order tables; T1, T2 hold N x M vector-type
  // elements each
  int fast = 0;
  const void* twN = nullptr;
  const void* twM = nullptr;
  // fast form, direction output: rho = r . z from the spectral coefficients
  // (Parseval: sum rhat^2 / (lambda + mu)) in the column pass, then the last
  // pass writes p_out = z + beta p_in (beta = rho_iter / rho_{iter-1}; p_out
  // = z at iter 0) instead of z and the dots
  int spectral = 0;
  int iter = 0;
  const void* p_in = nullptr;
  void* p_out = nullptr;
  // with spectral and a fused head: the iterate correction (T); the last
  // pass adds alpha_{iter-1} p_in to it while it reads p_in for the new
  // direction, and, if the rho step found convergence (FL_DPEND), does only
  // that
  void* d = nullptr;
  // the row DCT-II of r already ran, fused with the CG update that produced r
  // (launch_cg_update_fast); the prologue then only tests convergence
  int fused_head = 0;
  int small_tiles = 0;        // 16-bit products: 128 x 128 tiles even where 256 x 256 divide
  LaunchLog* log = nullptr;   // nullable: per-launch events
};
int launch_precond_fast(const PrecondArgs& a, hipStream_t s);
// Blocks of the fast form's row passes over an N x M image.
int fct_row_blocks(int64_t N, int64_t M);
// The CG update of iteration iter fused with the first pass of the next
// preconditioner application: alpha (and the FP16 input scale from the bound
// ||r|| + |alpha| ||q|| on the new residual) in one block, then per row
// r -= alpha q and the DCT-II of the new r into a.T1; partials ||r||^2,
// sum r zero padded to nparts_out.  The iterate update d += alpha p is left
// to the application's last pass (PrecondArgs::d), which reads p anyway.
// Returns the row-pass grid.
template <class T>
int launch_cg_update_fast(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter,
                          int nparts_out, hipStream_t s);

// ---- augmented (U, V^v, V^h) solve ------------------------------------------
template <class T>
struct AugVec {
  T* u; T* v; T* h;   // U block and the two slack blocks, Np x ld each
};
template <class T>
struct AugArgs {
  int64_t N, M, Np, ld;
  double tau, delta;
  const T* Gv; const T* Gh; const T* Cv; const T* Ch;
  T* dv; T* dh;       // C^2 / W on every edge (0 where no edge)
  DevState st;
};
enum AugOp : int {
  AUG_WEIGHTS = 0,    // x: weights, F_delta and L1 into SC_H, SC_L1
  AUG_RHS = 1,        // x = start (i0 = init), y = b; ||b||^2, tolerance d0
  AUG_START = 2,      // ||b||^2 over i0 partials, tolerance d0
  AUG_RESID = 3,      // x, y = b -> z = r; i0 = check_done
  AUG_VPRECOND = 4,   // x = r -> y = z (slack blocks)
  AUG_PUPDATE = 5,    // x = z, y = p; i0 = iter, i1 / i2 = partials of z.r (U / slack)
  AUG_APPLY = 6,      // x = p -> y = q
  AUG_AXPY = 7,       // x, y = r, z = p, w = q; i0 = iter, i1 = p.q partials
  AUG_CENTER = 8,     // x.u -= mean
  AUG_CAND = 9,       // x -> y = candidate step of Theorem 3 (1 / L from SC_INVL)
  AUG_HVAL = 10,      // (prob:alt1) objective of x at the current weights -> sc[i0]
  AUG_GUARD = 11,     // x = y when sc[SC_SNEW] > sc[SC_SOLD] or i0 == 2; FL_GUARD
  AUG_INVL = 12       // 1 / L = 1 / (12 / tau + C_max^2 / delta) into SC_INVL
};
template <class T>
int aug_launch(int op, const AugArgs<T>& a, const AugVec<T>& x, const AugVec<T>& y,
               const AugVec<T>& z, const AugVec<T>& w, int i0, int i1, int i2, double d0,
               hipStream_t s);
bool fct_supported(int64_t n);
size_t fct_table_bytes(int64_t n, int elem);
// general: the layout of the sides that are not powers of two (fctg.hip),
// also where one side of such a plan is a power of two
void launch_fct_tables(int elem, int64_t n, void* tw, double* eig, hipStream_t s,
                       bool general = false);
// Fast form for plans whose sides are not both powers of two (fctg.hip):
// each side n a multiple of 8 whose half has no prime factor above 5,
// n / 2 <= 8192.  The plan's vectors keep their row stride Mp and T1 / T2
// span the padded Np x Mp.
bool fctg_supported(int64_t n);
int fctg_row_blocks(int64_t N, int64_t M);
void launch_fctg_tables(int elem, int64_t n, void* tw, double* eig, hipStream_t s);
int launch_precond_fastg(const PrecondArgs& a, hipStream_t s);
template <class T>
int launch_cg_update_fastg(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter,
                           int nparts_out, hipStream_t s);
// pieces of the power-of-two passes that the general sizes share
template <class T>
void launch_transpose_any(const T* in, int64_t rows, int64_t cols, T* out, const int32_t* done,
                          hipStream_t s);
// the transpose back with rho, beta and the convergence test in its first block
template <class T>
void launch_transpose_rho(const T* in, int64_t rows, int64_t cols, T* out, DevState st, int n,
                          int iter, int f16, int nparts_rr, hipStream_t s);
void launch_fct_fold_partials(DevState st, int n, hipStream_t s);
void launch_cg_alpha(DevState st, int nparts_pq, int iter, int f16, double npix, hipStream_t s);
// Returns the number of partials written by the last product (z.r etc.).
int launch_precond(const PrecondArgs& a, hipStream_t s);
// Grouped preconditioner over the tiles of a batch (operand kind of the
// batch); starts[g] are the per-tile block prefixes of product g (4 x
// (ntiles + 1) entries, device), totals[g] the grid sizes.
void launch_precond_batched(int kind, const void* tiles, const int32_t* starts, int ntiles,
                            const int* totals, int check_conv, const int32_t* st_start,
                            int st_total, hipStream_t s);
// Per-tile block counts of the four products (host side, for the prefixes).
void precond_blocks(int kind, int64_t Np, int64_t Mp, int out[4]);
void launch_basis(int kind, int64_t n, int64_t npad, void* P, void* Pt, void* eig_inv,
                  hipStream_t s);
void launch_fold_basis(int kind, int64_t n, int64_t hp, void* Pe, void* Pet, void* Po, void* Pot,
                       void* eig, hipStream_t s);
void launch_fold_prologue(DevState st, int nparts_rr, int check_conv, int want_scale, int64_t npix,
                          hipStream_t s);
template <class TI, class TO>
void launch_fold_rows(const TI* in, int64_t ldin, int64_t n, int64_t rows_valid, int64_t rows,
                      TO* out, int64_t hp, const double* dscale, const int32_t* done,
                      hipStream_t s);
template <class OT>
void launch_unfold_rows(const OT* eo, int64_t ld, int64_t N, int64_t hNp, int64_t Np, OT* out,
                        const int32_t* done, hipStream_t s);
template <class T>
int launch_unfold_cols_dots(const T* zeo, int64_t hMp, int64_t N, int64_t M, int64_t Np, int64_t ld,
                            T* z, const T* r, const T* q, double zscale, const double* dscale,
                            DevState st, hipStream_t s);

}  // namespace irlsu
