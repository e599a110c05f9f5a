// Host side of the irlsu C ABI: plans (DCT bases and eigenvalues), the
// workspace carve-up, input validation and the IRLS + PCG driver.
//
// Per IRLS iteration (Algorithm 1): one weight step, then PCG (Algorithm 2):
//   init:  r = b - A u (FP64 u) | G1..G4 preconditioner (G1 checks ||r||)
//   loop:  stencil (p = z + beta p, q = A p, p.q) | axpy (u += alpha p,
//          r -= alpha q, ||r||^2) | [true residual every T iterations] |
//          G1..G4 (stops when ||r|| <= tol ||b||)
// Every scalar (rho, alpha, beta, norms) lives on the device and is reduced in
// a fixed order inside the consuming kernel's prologue; the host only reads
// the convergence flag every poll_every iterations.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "kernels.hpp"

using namespace irlsu;

struct irlsu_plan {
  int64_t N = 0, M = 0, Np = 0, Mp = 0;
  irlsu_precision prec = IRLSU_F32;
  int kind = OK_F32;
  size_t elem = 4;    // vector element bytes
  size_t opsz = 4;    // preconditioner operand bytes
  void* PN = nullptr;
  void* PNt = nullptr;
  void* PM = nullptr;
  void* PMt = nullptr;
  double* eigN = nullptr;
  double* eigM = nullptr;
  size_t plan_bytes = 0;
  size_t ws_bytes = 0;
  int32_t* h_flags = nullptr;   // pinned
  double* h_sc = nullptr;       // pinned
  int device = 0;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum VecId { V_R, V_Z, V_P0, V_P1, V_Q, V_B, V_GV, V_GH, V_CV, V_CH, V_OV, V_OH, V_COUNT };

struct Layout {
  size_t u, vec[V_COUNT], t1, t2, t3, part, sc, fl, total;
};

Layout layout(const irlsu_plan* p) {
  Layout L;
  const size_t npx = (size_t)p->Np * (size_t)p->Mp;
  size_t off = 0;
  L.u = off;
  off = align_up(off + npx * sizeof(double));
  for (int v = 0; v < V_COUNT; ++v) {
    L.vec[v] = off;
    off = align_up(off + npx * p->elem);
  }
  L.t1 = off;
  off = align_up(off + npx * p->opsz);
  L.t2 = off;
  off = align_up(off + npx * p->opsz);
  L.t3 = off;
  off = align_up(off + npx * p->opsz);
  L.part = off;
  off = align_up(off + (size_t)kPartSlots * kMaxPartials * sizeof(double));
  L.sc = off;
  off = align_up(off + SC_COUNT * sizeof(double));
  L.fl = off;
  off = align_up(off + FL_COUNT * sizeof(int32_t));
  L.total = off;
  return L;
}

template <class T>
struct Ws {
  double* U;
  T* v[V_COUNT];
  void *T1, *T2, *T3;
  DevState st;
};

template <class T>
Ws<T> carve(const irlsu_plan* p, void* base) {
  const Layout L = layout(p);
  char* b = static_cast<char*>(base);
  Ws<T> w;
  w.U = reinterpret_cast<double*>(b + L.u);
  for (int v = 0; v < V_COUNT; ++v) w.v[v] = reinterpret_cast<T*>(b + L.vec[v]);
  w.T1 = b + L.t1;
  w.T2 = b + L.t2;
  w.T3 = b + L.t3;
  w.st.part = reinterpret_cast<double*>(b + L.part);
  w.st.sc = reinterpret_cast<double*>(b + L.sc);
  w.st.fl = reinterpret_cast<int32_t*>(b + L.fl);
  return w;
}

#define HIP_OK(expr)                                  \
  do {                                                \
    if ((expr) != hipSuccess) return IRLSU_ERR_HIP;   \
  } while (0)

irlsu_status last_launch() {
  return hipGetLastError() == hipSuccess ? IRLSU_OK : IRLSU_ERR_HIP;
}

bool is_mixed(irlsu_precision p) { return p == IRLSU_MIXED_BF16 || p == IRLSU_MIXED_F16; }

template <class T>
PrecondArgs precond_args(const irlsu_plan* pl, const Ws<T>& W, const T* r, T* z, const T* q,
                         int check_conv, int nparts_rr) {
  PrecondArgs a;
  a.kind = pl->kind;
  a.N = pl->N;
  a.M = pl->M;
  a.Np = pl->Np;
  a.Mp = pl->Mp;
  a.PN = pl->PN;
  a.PNt = pl->PNt;
  a.PM = pl->PM;
  a.PMt = pl->PMt;
  a.eigN = pl->eigN;
  a.eigM = pl->eigM;
  a.T1 = W.T1;
  a.T2 = W.T2;
  a.T3 = W.T3;
  a.r = r;
  a.z = z;
  a.q = q;
  a.scale = 1.0;
  a.check_conv = check_conv;
  a.nparts_rr = nparts_rr;
  a.st = W.st;
  return a;
}

template <class T>
StencilArgs<T> stencil_base(const irlsu_plan* pl, const T* Ov, const T* Oh, DevState st) {
  StencilArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.Ov = Ov;
  a.Oh = Oh;
  a.N = pl->N;
  a.M = pl->M;
  a.Np = pl->Np;
  a.ld = pl->Mp;
  a.st = st;
  return a;
}

// Axpy grid: exactly as many blocks as the residual stencil, so that both
// producers of the ||r||^2 partials write the same count.
int stencil_blocks(const irlsu_plan* pl) {
  int rows = 0;
  const dim3 g = stencil_grid(pl->Np, pl->Mp, &rows);
  return (int)(g.x * g.y);
}

template <class T>
irlsu_status read_back(irlsu_plan* pl, const Ws<T>& W, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(pl->h_flags, W.st.fl, FL_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(pl->h_sc, W.st.sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return IRLSU_OK;
}

template <class T>
irlsu_status unwrap_impl(irlsu_plan* pl, const T* X, int64_t ldx, const T* w, const T* Cv,
                         int64_t ldcv, const T* Ch, int64_t ldch, const T* U0,
                         const irlsu_params& prm, T* Uout, int64_t ldu, void* ws,
                         irlsu_stats* stats, hipStream_t s) {
  const Ws<T> W = carve<T>(pl, ws);
  const int64_t N = pl->N, M = pl->M, Np = pl->Np, ld = pl->Mp;
  const size_t npx = (size_t)Np * (size_t)ld;
  DevState st = W.st;

  HIP_OK(hipMemsetAsync(st.fl, 0, FL_COUNT * sizeof(int32_t), s));
  HIP_OK(hipMemsetAsync(st.sc, 0, SC_COUNT * sizeof(double), s));
  for (int v = 0; v < V_COUNT; ++v) HIP_OK(hipMemsetAsync(W.v[v], 0, npx * sizeof(T), s));

  SetupArgs<T> sa;
  sa.X = X;
  sa.ldx = ldx;
  sa.w = w;
  sa.Cv = Cv;
  sa.ldcv = ldcv;
  sa.Ch = Ch;
  sa.ldch = ldch;
  sa.U0 = U0;
  sa.ldu0 = ldu;
  sa.N = N;
  sa.M = M;
  sa.Np = Np;
  sa.ld = ld;
  sa.Gv = W.v[V_GV];
  sa.Gh = W.v[V_GH];
  sa.Cv_out = W.v[V_CV];
  sa.Ch_out = W.v[V_CH];
  sa.U = W.U;
  sa.flags = st.fl + FL_INPUT;
  launch_setup<T>(sa, s);
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  irlsu_status rs = read_back(pl, W, s);
  if (rs != IRLSU_OK) return rs;
  if (pl->h_flags[FL_INPUT] & 1) return IRLSU_ERR_NONFINITE;
  if (pl->h_flags[FL_INPUT] & 2) return IRLSU_ERR_BAD_WEIGHTS;

  const int flexible = prm.flexible < 0 ? (is_mixed(pl->prec) ? 1 : 0) : prm.flexible;
  const double tol2 = prm.pcg_rtol * prm.pcg_rtol;
  const int nvec = stencil_blocks(pl);
  const bool want_obj = stats != nullptr || prm.l1_target > 0.0;
  T* P[2] = {W.v[V_P0], W.v[V_P1]};

  WeightsArgs<T> wa;
  wa.U = W.U;
  wa.Gv = W.v[V_GV];
  wa.Gh = W.v[V_GH];
  wa.Cv = W.v[V_CV];
  wa.Ch = W.v[V_CH];
  wa.Ov = W.v[V_OV];
  wa.Oh = W.v[V_OH];
  wa.b = W.v[V_B];
  wa.eps = prm.eps;
  wa.Np = Np;
  wa.ld = ld;
  wa.st = st;

  irlsu_status overall = IRLSU_OK;
  int pcg_total = 0, done_iters = 0;
  bool target_hit = false;
  for (int k = 0; k < prm.irls_iters; ++k) {
    const int nw = launch_weights<T>(wa, s);
    launch_finalize_weights(st, nw, nullptr, tol2, s);
    if (want_obj) {
      rs = read_back(pl, W, s);
      if (rs != IRLSU_OK) return rs;
      if (stats && k < IRLSU_MAX_IRLS) {
        stats->iter[k].L1 = pl->h_sc[SC_L1];
        stats->iter[k].H = pl->h_sc[SC_H];
      }
      if (prm.l1_target > 0.0 && pl->h_sc[SC_L1] <= prm.l1_target) {
        target_hit = true;
        break;
      }
    }
    // ---- PCG (Algorithm 2), warm start from the current U ----
    StencilArgs<T> ra = stencil_base<T>(pl, W.v[V_OV], W.v[V_OH], st);
    ra.u = W.U;
    ra.b = W.v[V_B];
    ra.r = W.v[V_R];
    ra.check_done = 0;
    launch_stencil<T>(ST_RESID, ra, s);
    PrecondArgs pa = precond_args<T>(pl, W, W.v[V_R], W.v[V_Z], flexible ? W.v[V_Q] : nullptr, 1,
                                     nvec);
    const int nprec = launch_precond(pa, s);
    int l = 0;
    for (l = 0; l < prm.pcg_max; ++l) {
      StencilArgs<T> fa = stencil_base<T>(pl, W.v[V_OV], W.v[V_OH], st);
      fa.z = W.v[V_Z];
      fa.p_in = P[(l + 1) & 1];
      fa.p_out = P[l & 1];
      fa.q = W.v[V_Q];
      fa.iter = l;
      fa.flexible = flexible;
      fa.nparts_prec = nprec;
      fa.nparts_res = nvec;
      fa.check_done = 1;
      const int npq = launch_stencil<T>(ST_FUSED, fa, s);
      AxpyArgs<T> xa;
      xa.u = W.U;
      xa.r = W.v[V_R];
      xa.p = P[l & 1];
      xa.q = W.v[V_Q];
      xa.n = (int64_t)npx;
      xa.nparts_pq = npq;
      xa.iter = l;
      xa.st = st;
      launch_axpy<T>(xa, s, nvec);
      if (prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max) {
        ra.check_done = 1;
        launch_stencil<T>(ST_RESID, ra, s);
      }
      if (l + 1 < prm.pcg_max) launch_precond(pa, s);
      if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
      if (prm.poll_every > 0 && (l + 1) % prm.poll_every == 0) {
        HIP_OK(hipMemcpyAsync(pl->h_flags, st.fl, FL_COUNT * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (pl->h_flags[FL_DONE]) break;
      }
    }
    launch_finalize_rr(st, nvec, s);
    rs = read_back(pl, W, s);
    if (rs != IRLSU_OK) return rs;
    const int iters = pl->h_flags[FL_ITERS];
    irlsu_status solve_st = IRLSU_OK;
    if (pl->h_flags[FL_STATUS] & 1) solve_st = IRLSU_ERR_BREAKDOWN;
    else if (!pl->h_flags[FL_DONE] && iters >= prm.pcg_max) solve_st = IRLSU_NOT_CONVERGED;
    if (stats && k < IRLSU_MAX_IRLS) {
      stats->iter[k].pcg_iters = iters;
      stats->iter[k].status = solve_st;
      const double bb = pl->h_sc[SC_BB];
      stats->iter[k].relres = bb > 0 ? std::sqrt(pl->h_sc[SC_RR] / bb) : 0.0;
    }
    pcg_total += iters;
    done_iters = k + 1;
    if (solve_st == IRLSU_ERR_BREAKDOWN) return IRLSU_ERR_BREAKDOWN;
    if (solve_st == IRLSU_NOT_CONVERGED) overall = IRLSU_NOT_CONVERGED;
    launch_mean_removal(W.U, N, M, ld, st, s);
  }
  if (want_obj) {
    const int nw = launch_weights<T>(wa, s);
    launch_finalize_weights(st, nw, nullptr, tol2, s);
    rs = read_back(pl, W, s);
    if (rs != IRLSU_OK) return rs;
    if (prm.l1_target > 0.0 && pl->h_sc[SC_L1] <= prm.l1_target) target_hit = true;
  }
  if (stats) {
    stats->irls_done = done_iters;
    stats->pcg_total = pcg_total;
    stats->target_hit = target_hit ? 1 : 0;
    stats->L1_final = pl->h_sc[SC_L1];
    stats->H_final = pl->h_sc[SC_H];
    stats->status = overall;
    if (done_iters < IRLSU_MAX_IRLS) {
      stats->iter[done_iters].L1 = pl->h_sc[SC_L1];
      stats->iter[done_iters].H = pl->h_sc[SC_H];
    }
  }
  launch_copy_out<T>(W.U, ld, Uout, ldu, N, M, s);
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  if (stats) HIP_OK(hipStreamSynchronize(s));
  return overall;
}

irlsu_status check_ws(const irlsu_plan* pl, const void* ws, size_t bytes) {
  if (!ws || bytes < pl->ws_bytes) return IRLSU_ERR_WORKSPACE;
  return IRLSU_OK;
}

}  // namespace

extern "C" {

const char* irlsu_status_string(irlsu_status st) {
  switch (st) {
    case IRLSU_OK: return "IRLSU_OK";
    case IRLSU_NOT_CONVERGED: return "IRLSU_NOT_CONVERGED: a PCG solve reached pcg_max";
    case IRLSU_ERR_INVALID_ARG: return "IRLSU_ERR_INVALID_ARG: null pointer, bad stride or parameter";
    case IRLSU_ERR_SHAPE: return "IRLSU_ERR_SHAPE: N and M must be >= 2 and match the plan";
    case IRLSU_ERR_NONFINITE: return "IRLSU_ERR_NONFINITE: NaN or Inf in the input";
    case IRLSU_ERR_BAD_WEIGHTS: return "IRLSU_ERR_BAD_WEIGHTS: weights must be > 0";
    case IRLSU_ERR_BREAKDOWN: return "IRLSU_ERR_BREAKDOWN: p^T A p <= 0 in PCG";
    case IRLSU_ERR_HIP: return "IRLSU_ERR_HIP: a HIP runtime call failed";
    case IRLSU_ERR_OOM: return "IRLSU_ERR_OOM: device allocation failed";
    case IRLSU_ERR_UNSUPPORTED: return "IRLSU_ERR_UNSUPPORTED: precision not supported";
    case IRLSU_ERR_WORKSPACE: return "IRLSU_ERR_WORKSPACE: workspace missing or too small";
  }
  return "IRLSU: unknown status";
}

irlsu_status irlsu_params_default(irlsu_params* p, irlsu_precision prec) {
  if (!p) return IRLSU_ERR_INVALID_ARG;
  if (prec < IRLSU_F64 || prec > IRLSU_MIXED_F16) return IRLSU_ERR_UNSUPPORTED;
  std::memset(p, 0, sizeof(*p));
  p->eps = 1e-3;
  p->pcg_rtol = prec == IRLSU_F64 ? 1e-8 : 1e-6;
  p->l1_target = 0.0;
  p->irls_iters = 20;
  p->pcg_max = 100;
  p->true_res_every = 32;
  p->poll_every = 4;
  p->flexible = -1;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_create(irlsu_plan** out, int64_t N, int64_t M, irlsu_precision prec,
                               void* stream) {
  if (!out) return IRLSU_ERR_INVALID_ARG;
  *out = nullptr;
  if (N < 2 || M < 2) return IRLSU_ERR_SHAPE;
  if (prec < IRLSU_F64 || prec > IRLSU_MIXED_F16) return IRLSU_ERR_UNSUPPORTED;
  if (N > (int64_t)1 << 20 || M > (int64_t)1 << 20) return IRLSU_ERR_SHAPE;
  irlsu_plan* p = new (std::nothrow) irlsu_plan;
  if (!p) return IRLSU_ERR_OOM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  p->N = N;
  p->M = M;
  p->prec = prec;
  p->Np = round_up(N, kTilePad);
  p->Mp = round_up(M, kTilePad);
  switch (prec) {
    case IRLSU_F64: p->kind = OK_F64; p->elem = 8; p->opsz = 8; break;
    case IRLSU_F32: p->kind = OK_F32; p->elem = 4; p->opsz = 4; break;
    case IRLSU_MIXED_BF16: p->kind = OK_BF16; p->elem = 4; p->opsz = 2; break;
    case IRLSU_MIXED_F16: p->kind = OK_F16; p->elem = 4; p->opsz = 2; break;
  }
  // the GEMM grids and the partial-sum table bound the supported size
  const int64_t tiles = (p->Np / 64) * (p->Mp / 64);
  if (tiles > kMaxPartials) {
    delete p;
    return IRLSU_ERR_SHAPE;
  }
  (void)hipGetDevice(&p->device);
  const bool share = (p->Np == p->Mp) && (N == M);
  const size_t bN = (size_t)p->Np * p->Np * p->opsz;
  const size_t bM = (size_t)p->Mp * p->Mp * p->opsz;
  bool ok = hipMalloc(&p->PN, bN) == hipSuccess && hipMalloc(&p->PNt, bN) == hipSuccess &&
            hipMalloc(&p->eigN, p->Np * sizeof(double)) == hipSuccess;
  if (ok && !share) {
    ok = hipMalloc(&p->PM, bM) == hipSuccess && hipMalloc(&p->PMt, bM) == hipSuccess &&
         hipMalloc(&p->eigM, p->Mp * sizeof(double)) == hipSuccess;
  }
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&p->h_flags), 256, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&p->h_sc), 512, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    irlsu_plan_destroy(p);
    return IRLSU_ERR_OOM;
  }
  if (share) {
    p->PM = p->PN;
    p->PMt = p->PNt;
    p->eigM = p->eigN;
  }
  p->plan_bytes = 2 * bN + p->Np * sizeof(double) + (share ? 0 : 2 * bM + p->Mp * sizeof(double));
  launch_basis(p->kind, N, p->Np, p->PN, p->PNt, p->eigN, s);
  if (!share) launch_basis(p->kind, M, p->Mp, p->PM, p->PMt, p->eigM, s);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    irlsu_plan_destroy(p);
    return IRLSU_ERR_HIP;
  }
  p->ws_bytes = layout(p).total;
  *out = p;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_destroy(irlsu_plan* p) {
  if (!p) return IRLSU_OK;
  const bool share = p->PM == p->PN;
  if (p->PN) (void)hipFree(p->PN);
  if (p->PNt) (void)hipFree(p->PNt);
  if (p->eigN) (void)hipFree(p->eigN);
  if (!share) {
    if (p->PM) (void)hipFree(p->PM);
    if (p->PMt) (void)hipFree(p->PMt);
    if (p->eigM) (void)hipFree(p->eigM);
  }
  if (p->h_flags) (void)hipHostFree(p->h_flags);
  if (p->h_sc) (void)hipHostFree(p->h_sc);
  delete p;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_info(const irlsu_plan* p, irlsu_plan_desc* out) {
  if (!p || !out) return IRLSU_ERR_INVALID_ARG;
  out->N = p->N;
  out->M = p->M;
  out->Np = p->Np;
  out->ld = p->Mp;
  out->precision = p->prec;
  out->elem_bytes = (int32_t)p->elem;
  out->workspace_bytes = p->ws_bytes;
  out->plan_bytes = p->plan_bytes;
  return IRLSU_OK;
}

size_t irlsu_workspace_bytes(const irlsu_plan* p) { return p ? p->ws_bytes : 0; }

irlsu_status irlsu_unwrap(irlsu_plan* plan, const void* X, int64_t ldx, const void* w,
                          const void* Cv, int64_t ldcv, const void* Ch, int64_t ldch,
                          const void* U0, const irlsu_params* params, void* U, int64_t ldu,
                          void* workspace, size_t workspace_bytes, irlsu_stats* stats,
                          void* stream) {
  if (!plan || !X || !U) return IRLSU_ERR_INVALID_ARG;
  if (ldx < plan->M || ldu < plan->M) return IRLSU_ERR_INVALID_ARG;
  if ((Cv == nullptr) != (Ch == nullptr)) return IRLSU_ERR_INVALID_ARG;
  if (Cv && (ldcv < plan->M || ldch < plan->M - 1)) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  irlsu_params prm;
  if (params) {
    prm = *params;
  } else {
    irlsu_params_default(&prm, plan->prec);
  }
  if (!(prm.eps > 0.0) || !(prm.pcg_rtol >= 0.0) || prm.irls_iters < 0 || prm.pcg_max < 1 ||
      prm.true_res_every < 0 || prm.poll_every < 0)
    return IRLSU_ERR_INVALID_ARG;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->elem == 8)
    return unwrap_impl<double>(plan, static_cast<const double*>(X), ldx,
                               static_cast<const double*>(w), static_cast<const double*>(Cv),
                               ldcv, static_cast<const double*>(Ch), ldch,
                               static_cast<const double*>(U0), prm, static_cast<double*>(U), ldu,
                               workspace, stats, s);
  return unwrap_impl<float>(plan, static_cast<const float*>(X), ldx,
                            static_cast<const float*>(w), static_cast<const float*>(Cv), ldcv,
                            static_cast<const float*>(Ch), ldch, static_cast<const float*>(U0),
                            prm, static_cast<float*>(U), ldu, workspace, stats, s);
}

irlsu_status irlsu_setup(const irlsu_plan* plan, const void* X, int64_t ldx, const void* w,
                         const void* Cv, int64_t ldcv, const void* Ch, int64_t ldch, void* Gv,
                         void* Gh, void* CvI, void* ChI, int32_t* flags, void* stream) {
  if (!plan || !X || !Gv || !Gh || !CvI || !ChI || !flags) return IRLSU_ERR_INVALID_ARG;
  if (ldx < plan->M || (Cv == nullptr) != (Ch == nullptr)) return IRLSU_ERR_INVALID_ARG;
  if (Cv && (ldcv < plan->M || ldch < plan->M - 1)) return IRLSU_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) {
    using T = decltype(tag);
    SetupArgs<T> a;
    a.X = static_cast<const T*>(X);
    a.ldx = ldx;
    a.w = static_cast<const T*>(w);
    a.Cv = static_cast<const T*>(Cv);
    a.ldcv = ldcv;
    a.Ch = static_cast<const T*>(Ch);
    a.ldch = ldch;
    a.U0 = nullptr;
    a.ldu0 = 0;
    a.N = plan->N;
    a.M = plan->M;
    a.Np = plan->Np;
    a.ld = plan->Mp;
    a.Gv = static_cast<T*>(Gv);
    a.Gh = static_cast<T*>(Gh);
    a.Cv_out = static_cast<T*>(CvI);
    a.Ch_out = static_cast<T*>(ChI);
    a.U = nullptr;
    a.flags = flags;
    launch_setup<T>(a, s);
  };
  if (plan->elem == 8) go(double{}); else go(float{});
  return last_launch();
}

irlsu_status irlsu_weights(const irlsu_plan* plan, double eps, const void* U, const void* Gv,
                           const void* Gh, const void* CvI, const void* ChI, void* Ov, void* Oh,
                           void* b, double* objectives, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (!plan || !U || !Gv || !Gh || !CvI || !ChI || !Ov || !Oh || !b || !objectives)
    return IRLSU_ERR_INVALID_ARG;
  if (!(eps > 0.0)) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    WeightsArgs<T> a;
    a.U = static_cast<const double*>(U);
    a.Gv = static_cast<const T*>(Gv);
    a.Gh = static_cast<const T*>(Gh);
    a.Cv = static_cast<const T*>(CvI);
    a.Ch = static_cast<const T*>(ChI);
    a.Ov = static_cast<T*>(Ov);
    a.Oh = static_cast<T*>(Oh);
    a.b = static_cast<T*>(b);
    a.eps = eps;
    a.Np = plan->Np;
    a.ld = plan->Mp;
    a.st = W.st;
    const int nw = launch_weights<T>(a, s);
    launch_finalize_weights(W.st, nw, objectives, 0.0, s);
  };
  if (plan->elem == 8) go(double{}); else go(float{});
  return last_launch();
}

irlsu_status irlsu_operator(const irlsu_plan* plan, const void* Ov, const void* Oh, const void* p,
                            void* q, double* pq, void* workspace, size_t workspace_bytes,
                            void* stream) {
  if (!plan || !Ov || !Oh || !p || !q) return IRLSU_ERR_INVALID_ARG;
  if (p == q) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    StencilArgs<T> a = stencil_base<T>(plan, static_cast<const T*>(Ov), static_cast<const T*>(Oh),
                                       W.st);
    a.p_in = static_cast<const T*>(p);
    a.q = static_cast<T*>(q);
    a.check_done = 0;
    const int n = launch_stencil<T>(ST_APPLY, a, s);
    if (pq) launch_reduce_to(W.st, PR_PQ, n, pq, s);
  };
  if (plan->elem == 8) go(double{}); else go(float{});
  return last_launch();
}

irlsu_status irlsu_precond(const irlsu_plan* plan, const void* r, void* z, double* rz,
                           void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !r || !z || r == z) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) -> irlsu_status {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    HIP_OK(hipMemsetAsync(W.st.fl, 0, FL_COUNT * sizeof(int32_t), s));
    PrecondArgs a = precond_args<T>(plan, W, static_cast<const T*>(r), static_cast<T*>(z), nullptr,
                                    0, 0);
    const int n = launch_precond(a, s);
    if (rz) launch_reduce_to(W.st, PR_ZR, n, rz, s);
    return IRLSU_OK;
  };
  st = plan->elem == 8 ? go(double{}) : go(float{});
  if (st != IRLSU_OK) return st;
  return last_launch();
}

}  // extern "C"
