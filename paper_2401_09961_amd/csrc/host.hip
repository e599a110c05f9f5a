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
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "tune.hpp"

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
  // fast preconditioner (power-of-two N and M): twiddle tables
  int fast = 0;
  void *twN = nullptr, *twM = nullptr;
  // timing aid: events of one armed PCG iteration (irlsu_profile_arm)
  int prof_k = -1, prof_l = -1;
  LaunchLog* prof = nullptr;
  // tuned launch shapes (0: the default rules): stencil band rows, blocks of
  // the CG update, 128 x 128 product tiles for 16-bit operands
  int tune_rows = 0, tune_update = 0, tune_small = 0;
  // stream on which PCG iterations are captured into graphs (non-blocking,
  // default priority); null when it could not be created
  hipStream_t cap_stream = nullptr;
  // events of the convergence polls read one block behind (null: each poll
  // synchronises the stream)
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  // folded preconditioner (even N and M)
  int folded = 0;
  int64_t hNp = 0, hMp = 0;
  void *PeN = nullptr, *PeNt = nullptr, *PoN = nullptr, *PoNt = nullptr;
  void *PeM = nullptr, *PeMt = nullptr, *PoM = nullptr, *PoMt = nullptr;
  double *eigNf = nullptr, *eigMf = nullptr;
};

struct irlsu_batch {
  int32_t ntiles = 0;
  irlsu_precision prec = IRLSU_MIXED_BF16;
  int kind = OK_BF16;
  size_t opsz = 2;                 // preconditioner operand / intermediate bytes
  std::vector<int> fast;           // per tile: fast-form preconditioner (sides powers of two)
  // twiddle and FP64 eigenvalue tables per side length of the fast tiles
  std::map<int64_t, int> fast_side_index;
  std::vector<void*> tw;
  std::vector<double*> eigf;
  std::vector<int64_t> N, M, Np, Mp;
  // basis tables per distinct side length
  std::map<int64_t, int> side_index;
  std::vector<void*> P, Pt;
  std::vector<double*> eig;
  // per-tile grids and partial ranges
  std::vector<int32_t> st_gx, st_rows, st_nblk, g4_nparts, part_off;
  int32_t st_total = 0;
  int g_total[4] = {0, 0, 0, 0};
  int32_t* d_st_start = nullptr;   // ntiles + 1
  int32_t* d_g_start = nullptr;    // 4 (ntiles + 1)
  void* d_tiles = nullptr;         // BatchTile<float>[ntiles]
  void* h_tiles = nullptr;         // pinned staging of the table
  int32_t* h_flags = nullptr;      // pinned, ntiles * FL_COUNT
  double* h_sc = nullptr;          // pinned, ntiles * SC_COUNT
  size_t ws_bytes = 0;
  std::vector<size_t> tile_off;    // workspace offset of each tile's vectors
  size_t part_off_bytes = 0, sc_off = 0, fl_off = 0;
  hipStream_t cap_stream = nullptr;  // capture stream of the PCG graphs (null: direct launches)
  hipEvent_t poll_ev[2] = {nullptr, nullptr};  // polls read one block behind (null: synchronous)
};

// ---- Scratch of the operator without allocation -------------------------
// irlsu_operator_noalloc keeps the per-block partial sums of p . q in this
// file-scope device array instead of a workspace: slot PR_PQ of a
// partial-sum table with kNoAllocParts entries per slot (96 KiB).  Every
// GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the name itself is a host-side stand-in).
constexpr int kNoAllocParts = 4096;
constexpr int kNoAllocSlots = PR_PQ + 1;
static __device__ __align__(256) double scratch[kNoAllocSlots * kNoAllocParts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current:
// resolved once per device (at plan creation), then read from the table.
double* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

// Allocation-failure hook of irlsu_test_fail_alloc: while armed (>= 0) it
// counts down the device and pinned allocations of plan and batch creation
// and fails the one it reaches zero on, as an out-of-memory device would.
int g_fail_alloc_at = -1;

bool fail_this_alloc() {
  if (g_fail_alloc_at < 0) return false;
  if (g_fail_alloc_at-- == 0) return true;
  return false;
}

hipError_t dev_malloc(void** ptr, size_t bytes) {
  if (fail_this_alloc()) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(ptr, bytes);
}

hipError_t pinned_malloc(void** ptr, size_t bytes, unsigned flags) {
  if (fail_this_alloc()) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(ptr, bytes, flags);
}

constexpr size_t kAlign = 256;
constexpr size_t kStagger = 4096;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum VecId { V_R, V_Z, V_P0, V_P1, V_Q, V_B, V_GV, V_GH, V_CV, V_CH, V_OV, V_OH, V_D, V_COUNT };

struct Layout {
  size_t u, lam, vec[V_COUNT], t1, t2, t3, zeo, part, sc, fl, total;
};

Layout layout(const irlsu_plan* p) {
  Layout L;
  const size_t npx = (size_t)p->Np * (size_t)p->Mp;
  size_t off = 0;
  L.u = off;
  off = align_up(off + npx * sizeof(double));
  L.lam = off;
  off = align_up(off + npx * sizeof(double));
  // each vector starts 4 KiB further along than the plain carve-up would put
  // it: vectors of 2^k bytes would otherwise all sit at the same offset
  // modulo the HBM interleave, and the kernels that stream three or four of
  // them at the same index lose about 3% of their bandwidth to that
  for (int v = 0; v < V_COUNT; ++v) {
    L.vec[v] = off;
    off = align_up(off + npx * p->elem) + kStagger;
  }
  // preconditioner intermediates: dense form Np x Mp each; folded form two
  // ping-pong buffers of 2 hNp x 2 hMp and an Np x 2 hMp vector-type buffer
  // (fast form: two N x M buffers of the vector type)
  const size_t inter = p->folded ? (size_t)(2 * p->hNp) * (size_t)(2 * p->hMp) : npx;
  const size_t isz = p->opsz;
  L.t1 = off;
  off = align_up(off + inter * isz) + kStagger;
  L.t2 = off;
  off = align_up(off + inter * isz) + kStagger;
  L.t3 = off;
  off = align_up(off + ((p->folded || p->fast) ? 0 : npx) * p->opsz);
  L.zeo = off;
  off = align_up(off + (p->folded ? (size_t)p->Np * (size_t)(2 * p->hMp) : 0) * p->elem);
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
  double* lam;
  T* v[V_COUNT];
  void *T1, *T2, *T3, *ZEO;
  DevState st;
};

template <class T>
Ws<T> carve(const irlsu_plan* p, void* base) {
  const Layout L = layout(p);
  char* b = static_cast<char*>(base);
  Ws<T> w;
  w.U = reinterpret_cast<double*>(b + L.u);
  w.lam = reinterpret_cast<double*>(b + L.lam);
  for (int v = 0; v < V_COUNT; ++v) w.v[v] = reinterpret_cast<T*>(b + L.vec[v]);
  w.T1 = b + L.t1;
  w.T2 = b + L.t2;
  w.T3 = b + L.t3;
  w.ZEO = b + L.zeo;
  w.st.part = reinterpret_cast<double*>(b + L.part);
  w.st.sc = reinterpret_cast<double*>(b + L.sc);
  w.st.fl = reinterpret_cast<int32_t*>(b + L.fl);
  w.st.off = 0;
  w.st.stride = 0;
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
  a.check_conv = check_conv;
  a.nparts_rr = nparts_rr;
  a.st = W.st;
  a.folded = pl->folded;
  a.hNp = pl->hNp;
  a.hMp = pl->hMp;
  a.PeN = pl->PeN;
  a.PeNt = pl->PeNt;
  a.PoN = pl->PoN;
  a.PoNt = pl->PoNt;
  a.PeM = pl->PeM;
  a.PeMt = pl->PeMt;
  a.PoM = pl->PoM;
  a.PoMt = pl->PoMt;
  a.eigNf = pl->eigNf;
  a.eigMf = pl->eigMf;
  a.ZEO = W.ZEO;
  a.fast = pl->fast;
  a.twN = pl->twN;
  a.twM = pl->twM;
  a.small_tiles = pl->tune_small;
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
  a.rows = pl->tune_rows;
  a.st = st;
  return a;
}

// Blocks of the CG update (axpy): the tuned count, at most the stencil's
// (the consumers read that many ||r||^2 partials, zero padded).
int update_blocks(const irlsu_plan* pl, int nvec) {
  if (pl->tune_update > 0) return std::min(pl->tune_update, nvec);
  return axpy_blocks(nvec);
}

// Blocks of the stencil (also the partial count of the residual producers).
int stencil_blocks(const irlsu_plan* pl) {
  int rows = 0;
  const dim3 g = stencil_grid(pl->Np, pl->Mp, &rows, pl->tune_rows);
  return (int)(g.x * g.y);
}

template <class T>
irlsu_status read_back(irlsu_plan* pl, const Ws<T>& W, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(pl->h_flags, W.st.fl, FL_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(pl->h_sc, W.st.sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return IRLSU_OK;
}

// Captured graphs of PCG iterations, by variant key, for one solve.  The
// launches are captured on the plan's own capture stream (the caller's may
// be the legacy default stream, which cannot be captured) and replayed on
// the caller's.  Nothing but kernel launches is captured.
class PcgGraphs {
 public:
  explicit PcgGraphs(hipStream_t cap) : cap_(cap) {}
  ~PcgGraphs() {
    for (auto& e : exec_)
      if (e.second) (void)hipGraphExecDestroy(e.second);
  }
  bool ok() const { return cap_ != nullptr; }
  template <class F>
  irlsu_status launch(uint64_t key, F&& record, hipStream_t s) {
    auto it = exec_.find(key);
    if (it == exec_.end()) {
      hipStream_t q = cap_;
      if (hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return IRLSU_ERR_HIP;
      record(q);
      hipGraph_t g = nullptr;
      const hipError_t e1 = hipStreamEndCapture(q, &g);
      if (e1 != hipSuccess || !g) {
        (void)hipGetLastError();
        return IRLSU_ERR_HIP;
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess || !ex) {
        (void)hipGetLastError();
        return IRLSU_ERR_HIP;
      }
      it = exec_.emplace(key, ex).first;
    }
    HIP_OK(hipGraphLaunch(it->second, s));
    return IRLSU_OK;
  }

 private:
  hipStream_t cap_;
  std::map<uint64_t, hipGraphExec_t> exec_;
};

// PCG (Algorithm 2) on D^T Omega D x = rhs with the Omega currently in the
// workspace, warm-started at x (FP64).  ||rhs||^2 and tol^2 must already be in
// SC_BB / SC_TOL2 and the flags cleared (finalize_weights / adjoint rhs).
// Default CG beta: flexible where 16-bit operands enter the MFMA products
// (dense / folded mixed plans: a preconditioner that is not quite linear or
// symmetric); plain for FP32 / FP64 plans and the fast form, whose
// transforms run in FP32 (its FP16 storage leaves the map close enough to
// linear that plain beta follows the flexible trajectory).
static int default_flexible(const irlsu_plan* pl) {
  return (is_mixed(pl->prec) && !pl->fast) ? 1 : 0;
}

template <class T>
irlsu_status pcg_solve(irlsu_plan* pl, const Ws<T>& W, double* x, const T* rhs,
                       const irlsu_params& prm, int flexible, int* iters_out, double* relres_out,
                       irlsu_status* solve_st, hipStream_t s, int irls_k = -1) {
  DevState st = W.st;
  const size_t npx = (size_t)pl->Np * (size_t)pl->Mp;
  const int nvec = stencil_blocks(pl);
  T* P[2] = {W.v[V_P0], W.v[V_P1]};
  // the solve accumulates its correction d (vector type) and adds it to x
  // (FP64) once at the end; the true-residual refresh uses x + d
  T* d = W.v[V_D];
  HIP_OK(hipMemsetAsync(d, 0, npx * sizeof(T), s));
  StencilArgs<T> ra = stencil_base<T>(pl, W.v[V_OV], W.v[V_OH], st);
  ra.u = x;
  ra.d = d;
  ra.b = rhs;
  ra.r = W.v[V_R];
  ra.check_done = 0;
  if (pl->fast && !flexible) ra.nparts_out = std::max(nvec, fct_row_blocks(pl->N, pl->M));
  launch_stencil<T>(ST_RESID, ra, s);
  PrecondArgs pa = precond_args<T>(pl, W, W.v[V_R], W.v[V_Z], flexible ? W.v[V_Q] : nullptr, 1,
                                   nvec);
  // Fast form with plain beta: rho = r . z comes from the spectral
  // coefficients (Parseval) in the column pass, and the last pass writes the
  // direction p_l = z_l + beta_l p_{l-1} itself; the stencil then only
  // applies the operator to p (it reads p and Omega instead of z, p_old and
  // Omega).
  const bool spectral = pl->fast && !flexible;
  // On that path the CG update of iteration l also runs fused with the next
  // application's first pass (launch_cg_update_fast), except where a
  // true-residual refresh follows it; the producers of ||r||^2 partials
  // (residual stencil, update, fused update) then write one common count.
  const int nrr = spectral ? std::max(nvec, fct_row_blocks(pl->N, pl->M)) : nvec;
  if (spectral) {
    pa.spectral = 1;
    pa.iter = 0;
    pa.p_out = P[0];
    pa.nparts_rr = nrr;
  }
  const int nprec = launch_precond(pa, s);
  // The launches of iteration l on stream q (no host work, no memset): the
  // loop issues them directly, or replays a captured graph of them.
  auto issue = [&](int l, LaunchLog* L, hipStream_t q) {
    StencilArgs<T> fa = stencil_base<T>(pl, W.v[V_OV], W.v[V_OH], st);
    fa.z = W.v[V_Z];
    fa.p_in = spectral ? P[l & 1] : P[(l + 1) & 1];
    fa.p_out = P[l & 1];
    fa.q = W.v[V_Q];
    fa.iter = l;
    fa.flexible = flexible;
    fa.nparts_prec = nprec;
    fa.nparts_res = nvec;
    fa.check_done = 1;
    fa.want_qq = spectral ? 1 : 0;
    const int npq = launch_stencil<T>(spectral ? ST_APPLY : ST_FUSED, fa, q);
    log_mark(L, IRLSU_LK_STENCIL, q);
    const bool refresh =
        prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max;
    if (spectral && !refresh && l + 1 < prm.pcg_max) {
      PrecondArgs fused = pa;
      fused.log = L;
      fused.iter = l + 1;
      fused.p_in = P[l & 1];
      fused.p_out = P[(l + 1) & 1];
      fused.fused_head = 1;
      fused.d = d;
      launch_cg_update_fast<T>(fused, W.v[V_R], W.v[V_Q], npq, l, nrr, q);
      launch_precond(fused, q);
      return;
    }
    AxpyArgs<T> xa;
    xa.u = x;
    xa.d = d;
    xa.r = W.v[V_R];
    xa.p = P[l & 1];
    xa.q = W.v[V_Q];
    xa.n = (int64_t)npx;
    xa.nparts_pq = npq;
    xa.nparts_out = nrr;
    xa.iter = l;
    xa.st = st;
    launch_axpy<T>(xa, q, update_blocks(pl, nvec));
    log_mark(L, IRLSU_LK_AXPY, q);
    if (refresh) {
      // the correction so far moves into the FP64 iterate before the true
      // residual is formed (d restarts at zero): d then only ever holds the
      // correction since the last refresh, so its rounding in the vector
      // type no longer bounds how far the residual can fall
      launch_commit<T>(x, d, (int64_t)npx, q, true);
      StencilArgs<T> rb = ra;
      rb.check_done = 1;
      launch_stencil<T>(ST_RESID, rb, q);
      log_mark(L, IRLSU_LK_RESIDUAL, q);
    }
    if (l + 1 < prm.pcg_max) {
      PrecondArgs pl_args = pa;
      pl_args.log = L;
      if (spectral) {
        pl_args.iter = l + 1;
        pl_args.p_in = P[l & 1];
        pl_args.p_out = P[(l + 1) & 1];
      }
      launch_precond(pl_args, q);
    }
  };
  // The loop runs in blocks of iterations, one per convergence poll.  A
  // block is replayed from a captured graph: every launch argument of
  // iteration l depends on l only through its parity, whether a
  // true-residual refresh follows it and whether it is the last (the
  // iteration count is kept on the device; beta = 0 at l = 0 only matters
  // to the fused stencil, whose first block runs directly), so a few graphs
  // serve a whole solve.  The poll of block b is read after block b + 1 has
  // been enqueued: the device never waits for the host, and a block enqueued
  // after convergence costs only kernels that return at once.
  PcgGraphs graphs(pl->cap_stream);
  const bool use_graph = prm.graph != 0 && graphs.ok();
  const int B = prm.poll_every > 0 ? prm.poll_every : 8;
  const bool ahead = pl->poll_ev[0] && pl->poll_ev[1];
  int pending = -1;
  for (int l0 = 0, blk = 0; l0 < prm.pcg_max; ++blk) {
    const int len = std::min(B, prm.pcg_max - l0);
    bool prof = false;
    for (int l = l0; l < l0 + len; ++l)
      prof = prof || (pl->prof && irls_k == pl->prof_k && l == pl->prof_l);
    if (!use_graph || prof || (!spectral && l0 == 0)) {
      for (int l = l0; l < l0 + len; ++l) {
        LaunchLog* L = (pl->prof && irls_k == pl->prof_k && l == pl->prof_l) ? pl->prof : nullptr;
        if (L) {
          L->n = 0;
          log_start(L, s);
        }
        issue(l, L, s);
      }
    } else {
      uint64_t key = (uint64_t)(l0 & 1) | ((uint64_t)len << 1);
      for (int i = 0; i < len; ++i) {
        const int l = l0 + i;
        const bool refresh =
            prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max;
        if (refresh) key |= (uint64_t)1 << (16 + i);
      }
      if (l0 + len >= prm.pcg_max) key |= (uint64_t)1 << 15;
      irlsu_status gs = graphs.launch(key, [&](hipStream_t q) {
        for (int l = l0; l < l0 + len; ++l) issue(l, nullptr, q);
      }, s);
      if (gs != IRLSU_OK) return gs;
    }
    if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
    l0 += len;
    if (prm.poll_every > 0) {
      int32_t* slot = pl->h_flags + (ahead ? (blk & 1) * FL_COUNT : 0);
      HIP_OK(hipMemcpyAsync(slot, st.fl, FL_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (!ahead) {
        HIP_OK(hipStreamSynchronize(s));
        if (slot[FL_DONE]) break;
        continue;
      }
      HIP_OK(hipEventRecord(pl->poll_ev[blk & 1], s));
      if (pending >= 0) {
        HIP_OK(hipEventSynchronize(pl->poll_ev[pending & 1]));
        if (pl->h_flags[(pending & 1) * FL_COUNT + FL_DONE]) break;
      }
      pending = blk;
    }
  }
  launch_finalize_rr(st, nrr, s);
  launch_commit<T>(x, d, (int64_t)npx, s);
  irlsu_status rs = read_back(pl, W, s);
  if (rs != IRLSU_OK) return rs;
  *iters_out = pl->h_flags[FL_ITERS];
  *solve_st = IRLSU_OK;
  if (pl->h_flags[FL_STATUS] & 1) *solve_st = IRLSU_ERR_BREAKDOWN;
  else if (!pl->h_flags[FL_DONE] && *iters_out >= prm.pcg_max) *solve_st = IRLSU_NOT_CONVERGED;
  const double bb = pl->h_sc[SC_BB];
  *relres_out = bb > 0 ? std::sqrt(pl->h_sc[SC_RR] / bb) : 0.0;
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

  const int flexible = prm.flexible < 0 ? default_flexible(pl) : prm.flexible;
  const double tol2 = prm.pcg_rtol * prm.pcg_rtol;
  const bool adaptive = prm.cg_schedule == IRLSU_CG_ADAPTIVE;
  const bool want_obj = stats != nullptr || prm.l1_target > 0.0 || adaptive;
  // iteration caps: fixed, or the Section 4.3 schedule (m_CG(-1) = m_CG(0))
  int cap = adaptive ? prm.cg_m0 : prm.pcg_max;
  int cap_prev = cap, cap_prev2 = cap;
  bool schedule_stop = false;

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
    wa.want_model = (adaptive && k > 0) ? 1 : 0;
    const int nw = launch_weights<T>(wa, s);
    launch_finalize_weights(st, nw, nullptr, tol2, s, wa.want_model);
    wa.want_model = 0;
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
    if (adaptive && k > 0) {
      const double s_old = pl->h_sc[SC_SOLD], s_new = pl->h_sc[SC_SNEW];
      const double delta = s_old > 0.0 ? (s_old - s_new) / s_old : 0.0;
      if (stats && k < IRLSU_MAX_IRLS) stats->iter[k].delta = delta;
      if (delta > prm.cg_eps_tol) {
        cap = cap_prev;
      } else if (cap_prev != cap_prev2) {
        schedule_stop = true;
        break;
      } else {
        cap = (int)std::ceil(prm.cg_alpha * (double)cap_prev);
      }
    }
    if (stats && k < IRLSU_MAX_IRLS) stats->iter[k].pcg_cap = cap;
    // ---- PCG (Algorithm 2), warm start from the current U ----
    int iters = 0;
    double relres = 0.0;
    irlsu_status solve_st = IRLSU_OK;
    irlsu_params pk = prm;
    pk.pcg_max = cap;
    rs = pcg_solve<T>(pl, W, W.U, W.v[V_B], pk, flexible, &iters, &relres, &solve_st, s, k);
    cap_prev2 = cap_prev;
    cap_prev = cap;
    if (rs != IRLSU_OK) return rs;
    if (stats && k < IRLSU_MAX_IRLS) {
      stats->iter[k].pcg_iters = iters;
      stats->iter[k].status = solve_st;
      stats->iter[k].relres = relres;
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
    stats->schedule_stop = schedule_stop ? 1 : 0;
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

// Adjoint solve on the state an irlsu_unwrap call left in the workspace:
// frozen weights at the final U, one PCG solve, edge gradients.
// Full implicit derivative of the Huber minimiser (the Hessian weights kappa
// replace Omega in the workspace; see adjoint.hip).
template <class T>
irlsu_status adjoint_implicit_impl(irlsu_plan* pl, const Ws<T>& W, const T* gU, int64_t ldg,
                                   const irlsu_params& prm, T* gCv, int64_t ldgcv, T* gCh,
                                   int64_t ldgch, T* gX, int64_t ldgx, irlsu_stats* stats,
                                   hipStream_t s) {
  const int64_t N = pl->N, M = pl->M, Np = pl->Np, ld = pl->Mp;
  const size_t npx = (size_t)Np * (size_t)ld;
  DevState st = W.st;
  T* Kv = W.v[V_OV];
  T* Kh = W.v[V_OH];
  launch_adjoint_hessian<T>(W.U, W.v[V_GV], W.v[V_GH], W.v[V_CV], W.v[V_CH], prm.eps, N, M, Np,
                            ld, Kv, Kh, s);
  launch_adjoint_rhs_implicit<T>(gU, ldg, N, M, Np, ld, Kv, Kh, W.v[V_B], st,
                                 prm.pcg_rtol * prm.pcg_rtol, s);
  HIP_OK(hipMemsetAsync(W.lam, 0, npx * sizeof(double), s));
  const int flexible = prm.flexible < 0 ? default_flexible(pl) : prm.flexible;
  int iters = 0;
  double relres = 0.0;
  irlsu_status solve_st = IRLSU_OK;
  irlsu_status rs = pcg_solve<T>(pl, W, W.lam, W.v[V_B], prm, flexible, &iters, &relres,
                                 &solve_st, s);
  if (rs != IRLSU_OK) return rs;
  if (solve_st == IRLSU_ERR_BREAKDOWN) return solve_st;
  launch_adjoint_lam_mean<T>(W.lam, N, M, ld, Kv, Kh, st, s);
  AdjEdgeArgs<T> ea;
  ea.U = W.U;
  ea.lam = W.lam;
  ea.Gv = W.v[V_GV];
  ea.Gh = W.v[V_GH];
  ea.Cv = W.v[V_CV];
  ea.Ch = W.v[V_CH];
  ea.eps = prm.eps;
  ea.N = N;
  ea.M = M;
  ea.ld = ld;
  ea.gCv = gCv;
  ea.ldgcv = ldgcv;
  ea.gCh = gCh;
  ea.ldgch = ldgch;
  ea.gX = gX;
  ea.ldgx = ldgx;
  ea.Kv = Kv;
  ea.Kh = Kh;
  ea.lam_mean = st.sc + SC_MEAN;
  launch_adjoint_edges<T>(ea, s);
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->pcg_total = iters;
    stats->status = solve_st;
    stats->iter[0].pcg_iters = iters;
    stats->iter[0].relres = relres;
    stats->iter[0].status = solve_st;
    HIP_OK(hipStreamSynchronize(s));
  }
  return solve_st;
}

template <class T>
irlsu_status adjoint_impl(irlsu_plan* pl, const T* gU, int64_t ldg, const irlsu_params& prm,
                          T* gCv, int64_t ldgcv, T* gCh, int64_t ldgch, T* gX, int64_t ldgx,
                          void* ws, irlsu_stats* stats, hipStream_t s, bool implicit) {
  const Ws<T> W = carve<T>(pl, ws);
  const int64_t N = pl->N, M = pl->M, Np = pl->Np, ld = pl->Mp;
  const size_t npx = (size_t)Np * (size_t)ld;
  DevState st = W.st;
  if (implicit)
    return adjoint_implicit_impl<T>(pl, W, gU, ldg, prm, gCv, ldgcv, gCh, ldgch, gX, ldgx, stats,
                                    s);
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
  launch_weights<T>(wa, s);
  launch_adjoint_rhs<T>(gU, ldg, N, M, Np, ld, W.v[V_B], st, prm.pcg_rtol * prm.pcg_rtol, s);
  HIP_OK(hipMemsetAsync(W.lam, 0, npx * sizeof(double), s));
  const int flexible = prm.flexible < 0 ? default_flexible(pl) : prm.flexible;
  int iters = 0;
  double relres = 0.0;
  irlsu_status solve_st = IRLSU_OK;
  irlsu_status rs = pcg_solve<T>(pl, W, W.lam, W.v[V_B], prm, flexible, &iters, &relres,
                                 &solve_st, s);
  if (rs != IRLSU_OK) return rs;
  if (solve_st == IRLSU_ERR_BREAKDOWN) return solve_st;
  AdjEdgeArgs<T> ea;
  ea.U = W.U;
  ea.lam = W.lam;
  ea.Gv = W.v[V_GV];
  ea.Gh = W.v[V_GH];
  ea.Cv = W.v[V_CV];
  ea.Ch = W.v[V_CH];
  ea.eps = prm.eps;
  ea.N = N;
  ea.M = M;
  ea.ld = ld;
  ea.gCv = gCv;
  ea.ldgcv = ldgcv;
  ea.gCh = gCh;
  ea.ldgch = ldgch;
  ea.gX = gX;
  ea.ldgx = ldgx;
  launch_adjoint_edges<T>(ea, s);
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->irls_done = 0;
    stats->pcg_total = iters;
    stats->status = solve_st;
    stats->iter[0].pcg_iters = iters;
    stats->iter[0].relres = relres;
    stats->iter[0].status = solve_st;
    HIP_OK(hipStreamSynchronize(s));
  }
  return solve_st;
}

// ---------------------------------------------------------------------------
// Batched tiles: every PCG phase is one grouped launch over all tiles.
// ---------------------------------------------------------------------------
constexpr int64_t kBatchPad = 256;
constexpr int kBatchVecs = 12;  // r z p0 p1 q b Gv Gh Cv Ch Ov Oh

size_t batch_tile_bytes(int64_t Np, int64_t Mp, size_t opsz) {
  const size_t npx = (size_t)Np * (size_t)Mp;
  return align_up(npx * sizeof(double)) + kBatchVecs * align_up(npx * sizeof(float)) +
         3 * align_up(npx * opsz);
}

// A tile runs the fast form when both sides are powers of two that the fast
// transforms take and that the batch padding leaves unpadded.
bool batch_tile_fast(int64_t N, int64_t M) {
  return fct_supported(N) && fct_supported(M) && N % kBatchPad == 0 && M % kBatchPad == 0;
}

struct TileWs {
  double* U;
  float* v[kBatchVecs];
  void *T1, *T2, *T3;
};

TileWs carve_tile(const irlsu_batch* b, void* base, int t) {
  const size_t npx = (size_t)b->Np[t] * (size_t)b->Mp[t];
  char* p = static_cast<char*>(base) + b->tile_off[t];
  TileWs w;
  w.U = reinterpret_cast<double*>(p);
  p += align_up(npx * sizeof(double));
  for (int v = 0; v < kBatchVecs; ++v) {
    w.v[v] = reinterpret_cast<float*>(p);
    p += align_up(npx * sizeof(float));
  }
  w.T1 = p;
  p += align_up(npx * b->opsz);
  w.T2 = p;
  p += align_up(npx * b->opsz);
  w.T3 = p;
  return w;
}

DevState tile_state(const irlsu_batch* b, void* base, int t) {
  char* p = static_cast<char*>(base);
  DevState st;
  st.part = reinterpret_cast<double*>(p + b->part_off_bytes);
  st.sc = reinterpret_cast<double*>(p + b->sc_off) + (size_t)t * SC_COUNT;
  st.fl = reinterpret_cast<int32_t*>(p + b->fl_off) + (size_t)t * FL_COUNT;
  st.off = b->part_off[t];
  st.stride = 0;
  return st;
}

irlsu_status batch_read_back(irlsu_batch* b, void* ws, hipStream_t s) {
  char* p = static_cast<char*>(ws);
  HIP_OK(hipMemcpyAsync(b->h_flags, p + b->fl_off, (size_t)b->ntiles * FL_COUNT * sizeof(int32_t),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(b->h_sc, p + b->sc_off, (size_t)b->ntiles * SC_COUNT * sizeof(double),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return IRLSU_OK;
}

irlsu_status unwrap_batched_impl(irlsu_batch* b, const irlsu_tile* tiles, const irlsu_params& prm,
                                 void* ws, irlsu_stats* stats, hipStream_t s) {
  const int nt = b->ntiles;
  char* base = static_cast<char*>(ws);
  HIP_OK(hipMemsetAsync(base + b->sc_off, 0, (size_t)nt * SC_COUNT * sizeof(double), s));
  HIP_OK(hipMemsetAsync(base + b->fl_off, 0, (size_t)nt * FL_COUNT * sizeof(int32_t), s));
  BatchTile<float>* ht = static_cast<BatchTile<float>*>(b->h_tiles);
  for (int t = 0; t < nt; ++t) {
    const TileWs w = carve_tile(b, ws, t);
    const size_t npx = (size_t)b->Np[t] * (size_t)b->Mp[t];
    for (int v = 0; v < kBatchVecs; ++v) HIP_OK(hipMemsetAsync(w.v[v], 0, npx * sizeof(float), s));
    const DevState st = tile_state(b, ws, t);
    SetupArgs<float> sa;
    sa.X = static_cast<const float*>(tiles[t].X);
    sa.ldx = tiles[t].ldx;
    sa.w = static_cast<const float*>(tiles[t].w);
    sa.Cv = static_cast<const float*>(tiles[t].Cv);
    sa.ldcv = tiles[t].ldcv;
    sa.Ch = static_cast<const float*>(tiles[t].Ch);
    sa.ldch = tiles[t].ldch;
    sa.U0 = nullptr;
    sa.ldu0 = 0;
    sa.N = b->N[t];
    sa.M = b->M[t];
    sa.Np = b->Np[t];
    sa.ld = b->Mp[t];
    sa.Gv = w.v[6];
    sa.Gh = w.v[7];
    sa.Cv_out = w.v[8];
    sa.Ch_out = w.v[9];
    sa.U = w.U;
    sa.flags = st.fl + FL_INPUT;
    launch_setup<float>(sa, s);
    BatchTile<float>& bt = ht[t];
    bt.N = b->N[t];
    bt.M = b->M[t];
    bt.Np = b->Np[t];
    bt.ld = b->Mp[t];
    bt.U = w.U;
    bt.r = w.v[0];
    bt.z = w.v[1];
    bt.p0 = w.v[2];
    bt.p1 = w.v[3];
    bt.q = w.v[4];
    bt.b = w.v[5];
    bt.Ov = w.v[10];
    bt.Oh = w.v[11];
    bt.st = st;
    bt.st_gx = b->st_gx[t];
    bt.st_rows = b->st_rows[t];
    bt.st_nblk = b->st_nblk[t];
    bt.g4_nparts = b->g4_nparts[t];
    bt.flexible_q = 0;
    bt.fast = b->fast[t];
    bt.T1 = w.T1;
    bt.T2 = w.T2;
    bt.T3 = w.T3;
    if (b->fast[t]) {
      bt.PN = bt.PNt = bt.PM = bt.PMt = nullptr;
      bt.eigN = bt.eigM = nullptr;
    } else {
      const int in = b->side_index.at(b->N[t]), im = b->side_index.at(b->M[t]);
      bt.PN = b->P[in];
      bt.PNt = b->Pt[in];
      bt.PM = b->P[im];
      bt.PMt = b->Pt[im];
      bt.eigN = b->eig[in];
      bt.eigM = b->eig[im];
    }
  }
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  irlsu_status rs = batch_read_back(b, ws, s);
  if (rs != IRLSU_OK) return rs;
  for (int t = 0; t < nt; ++t) {
    if (b->h_flags[t * FL_COUNT + FL_INPUT] & 1) return IRLSU_ERR_NONFINITE;
    if (b->h_flags[t * FL_COUNT + FL_INPUT] & 2) return IRLSU_ERR_BAD_WEIGHTS;
  }
  const int flexible = prm.flexible < 0 ? 1 : prm.flexible;
  for (int t = 0; t < nt; ++t) ht[t].flexible_q = flexible;
  // the fast-form tiles' own preconditioner launches (the single-image
  // passes on the tile's vectors; z with its dots folded into one partial)
  std::vector<PrecondArgs> fastp;
  for (int t = 0; t < nt; ++t) {
    if (!b->fast[t]) continue;
    const BatchTile<float>& bt = ht[t];
    PrecondArgs a{};
    a.kind = b->kind;
    a.N = bt.N;
    a.M = bt.M;
    a.Np = bt.Np;
    a.Mp = bt.ld;
    a.T1 = bt.T1;
    a.T2 = bt.T2;
    a.T3 = bt.T3;
    a.r = bt.r;
    a.z = bt.z;
    a.q = flexible ? bt.q : nullptr;
    a.check_conv = 1;
    a.nparts_rr = bt.st_nblk;
    a.st = bt.st;
    a.fast = 1;
    a.twN = b->tw[b->fast_side_index.at(bt.N)];
    a.twM = b->tw[b->fast_side_index.at(bt.M)];
    a.eigN = b->eigf[b->fast_side_index.at(bt.N)];
    a.eigM = b->eigf[b->fast_side_index.at(bt.M)];
    fastp.push_back(a);
  }
  HIP_OK(hipMemcpyAsync(b->d_tiles, b->h_tiles, (size_t)nt * sizeof(BatchTile<float>),
                        hipMemcpyHostToDevice, s));
  const BatchTile<float>* dt = static_cast<const BatchTile<float>*>(b->d_tiles);
  auto precond_all = [&](hipStream_t q) {
    launch_precond_batched(b->kind, dt, b->d_g_start, nt, b->g_total, 1, b->d_st_start,
                           b->st_total, q);
    for (const PrecondArgs& a : fastp) launch_precond(a, q);
  };
  const double tol2 = prm.pcg_rtol * prm.pcg_rtol;
  std::vector<int> pcg_total(nt, 0);
  std::vector<irlsu_status> overall(nt, IRLSU_OK);
  if (stats) std::memset(stats, 0, (size_t)nt * sizeof(irlsu_stats));

  auto weights_all = [&]() {
    for (int t = 0; t < nt; ++t) {
      const BatchTile<float>& bt = ht[t];
      const TileWs w = carve_tile(b, ws, t);
      WeightsArgs<float> wa;
      wa.U = w.U;
      wa.Gv = w.v[6];
      wa.Gh = w.v[7];
      wa.Cv = w.v[8];
      wa.Ch = w.v[9];
      wa.Ov = w.v[10];
      wa.Oh = w.v[11];
      wa.b = w.v[5];
      wa.eps = prm.eps;
      wa.Np = bt.Np;
      wa.ld = bt.ld;
      wa.st = bt.st;
      const int nw = launch_weights<float>(wa, s);
      launch_finalize_weights(bt.st, nw, nullptr, tol2, s);
    }
  };

  PcgGraphs graphs(b->cap_stream);
  const bool use_graph = prm.graph != 0 && graphs.ok();
  for (int k = 0; k < prm.irls_iters; ++k) {
    weights_all();
    if (stats) {
      rs = batch_read_back(b, ws, s);
      if (rs != IRLSU_OK) return rs;
      for (int t = 0; t < nt && k < IRLSU_MAX_IRLS; ++t) {
        stats[t].iter[k].L1 = b->h_sc[t * SC_COUNT + SC_L1];
        stats[t].iter[k].H = b->h_sc[t * SC_COUNT + SC_H];
      }
    }
    launch_stencil_batched<float>(ST_RESID, dt, b->d_st_start, nt, b->st_total, 0, flexible, 0, s);
    precond_all(s);
    // one PCG step over all tiles: grouped stencil, update, refresh,
    // preconditioner products; replayed from captured graphs for l >= 1
    // (the arguments depend on l only through its parity, the refresh and
    // the last iteration; iteration counts are kept on the device)
    auto step = [&](int l, hipStream_t q) {
      launch_stencil_batched<float>(ST_FUSED, dt, b->d_st_start, nt, b->st_total, l, flexible, 1,
                                    q);
      launch_axpy_batched<float>(dt, b->d_st_start, nt, b->st_total, l, q);
      if (prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max)
        launch_stencil_batched<float>(ST_RESID, dt, b->d_st_start, nt, b->st_total, l, flexible, 1,
                                      q);
      if (l + 1 < prm.pcg_max) precond_all(q);
    };
    // blocks of iterations between polls, as in the single-image loop
    // (graphs for the blocks after the first; each poll read one block
    // behind)
    const int B = prm.poll_every > 0 ? prm.poll_every : 8;
    const size_t fbytes = (size_t)nt * FL_COUNT * sizeof(int32_t);
    const bool ahead = b->poll_ev[0] && b->poll_ev[1];
    int pending = -1;
    for (int l0 = 0, blk = 0; l0 < prm.pcg_max; ++blk) {
      const int len = std::min(B, prm.pcg_max - l0);
      if (l0 == 0 || !use_graph) {
        for (int l = l0; l < l0 + len; ++l) step(l, s);
      } else {
        uint64_t key = (uint64_t)(l0 & 1) | ((uint64_t)len << 1);
        for (int i = 0; i < len; ++i) {
          const int l = l0 + i;
          if (prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max)
            key |= (uint64_t)1 << (16 + i);
        }
        if (l0 + len >= prm.pcg_max) key |= (uint64_t)1 << 15;
        rs = graphs.launch(key, [&](hipStream_t q) {
          for (int l = l0; l < l0 + len; ++l) step(l, q);
        }, s);
        if (rs != IRLSU_OK) return rs;
      }
      if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
      l0 += len;
      if (prm.poll_every > 0) {
        int32_t* slot = b->h_flags + (ahead ? (size_t)(blk & 1) * nt * FL_COUNT : 0);
        HIP_OK(hipMemcpyAsync(slot, base + b->fl_off, fbytes, hipMemcpyDeviceToHost, s));
        int32_t* check = nullptr;
        if (!ahead) {
          HIP_OK(hipStreamSynchronize(s));
          check = slot;
        } else {
          HIP_OK(hipEventRecord(b->poll_ev[blk & 1], s));
          if (pending >= 0) {
            HIP_OK(hipEventSynchronize(b->poll_ev[pending & 1]));
            check = b->h_flags + (size_t)(pending & 1) * nt * FL_COUNT;
          }
          pending = blk;
        }
        if (check) {
          bool all = true;
          for (int t = 0; t < nt; ++t) all = all && check[t * FL_COUNT + FL_DONE];
          if (all) break;
        }
      }
    }
    for (int t = 0; t < nt; ++t) launch_finalize_rr(ht[t].st, ht[t].st_nblk, s);
    rs = batch_read_back(b, ws, s);
    if (rs != IRLSU_OK) return rs;
    for (int t = 0; t < nt; ++t) {
      const int32_t* f = b->h_flags + t * FL_COUNT;
      const int iters = f[FL_ITERS];
      irlsu_status st = IRLSU_OK;
      if (f[FL_STATUS] & 1) st = IRLSU_ERR_BREAKDOWN;
      else if (!f[FL_DONE] && iters >= prm.pcg_max) st = IRLSU_NOT_CONVERGED;
      if (st == IRLSU_ERR_BREAKDOWN) return st;
      if (st == IRLSU_NOT_CONVERGED) overall[t] = st;
      pcg_total[t] += iters;
      if (stats && k < IRLSU_MAX_IRLS) {
        stats[t].iter[k].pcg_iters = iters;
        stats[t].iter[k].status = st;
        const double bb = b->h_sc[t * SC_COUNT + SC_BB];
        stats[t].iter[k].relres = bb > 0 ? std::sqrt(b->h_sc[t * SC_COUNT + SC_RR] / bb) : 0.0;
      }
    }
    for (int t = 0; t < nt; ++t) launch_mean_removal(ht[t].U, ht[t].N, ht[t].M, ht[t].ld, ht[t].st, s);
  }
  if (stats) {
    weights_all();
    rs = batch_read_back(b, ws, s);
    if (rs != IRLSU_OK) return rs;
  }
  irlsu_status worst = IRLSU_OK;
  for (int t = 0; t < nt; ++t) {
    launch_copy_out<float>(ht[t].U, ht[t].ld, static_cast<float*>(tiles[t].U), tiles[t].ldu,
                           ht[t].N, ht[t].M, s);
    if (overall[t] == IRLSU_NOT_CONVERGED) worst = IRLSU_NOT_CONVERGED;
    if (stats) {
      stats[t].irls_done = prm.irls_iters;
      stats[t].pcg_total = pcg_total[t];
      stats[t].status = overall[t];
      stats[t].L1_final = b->h_sc[t * SC_COUNT + SC_L1];
      stats[t].H_final = b->h_sc[t * SC_COUNT + SC_H];
      if (prm.irls_iters < IRLSU_MAX_IRLS) {
        stats[t].iter[prm.irls_iters].L1 = stats[t].L1_final;
        stats[t].iter[prm.irls_iters].H = stats[t].H_final;
      }
    }
  }
  if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
  if (stats) HIP_OK(hipStreamSynchronize(s));
  return worst;
}

// Stencil grids of the tiles (band rows: rows[t], 0 for the default rule),
// the partial-sum ranges they imply and the block prefix st_start; returns
// the partials the batch needs (at most kMaxPartials for a valid layout).
int64_t batch_grids(irlsu_batch* b, const std::vector<int>& rows, std::vector<int32_t>& st_start) {
  const int nt = b->ntiles;
  b->st_gx.assign(nt, 0);
  b->st_rows.assign(nt, 0);
  b->st_nblk.assign(nt, 0);
  b->g4_nparts.assign(nt, 0);
  b->part_off.assign(nt, 0);
  st_start.assign(nt + 1, 0);
  int64_t part = 0;
  for (int t = 0; t < nt; ++t) {
    const int64_t N = b->N[t], M = b->M[t], Np = b->Np[t], Mp = b->Mp[t];
    int r = 0;
    const dim3 g = stencil_grid(Np, Mp, &r, rows[t]);
    const int32_t nblk = (int32_t)(g.x * g.y);
    b->st_gx[t] = (int32_t)g.x;
    b->st_rows[t] = r;
    b->st_nblk[t] = nblk;
    // partials of z . r etc. that the stencil reads: the grouped dots kernel
    // writes one per stencil block; the fast passes fold theirs into one
    b->g4_nparts[t] = b->fast[t] ? 1 : nblk;
    int gb[4] = {0, 0, 0, 0};
    if (!b->fast[t]) precond_blocks(b->kind, Np, Mp, gb);
    int wrows = 1;
    const dim3 wg = weights_grid(Np, Mp, &wrows);
    const int32_t need = std::max({nblk, gb[3], (int32_t)(wg.x * wg.y),
                                   (int32_t)elementwise_blocks(Np * Mp),
                                   b->fast[t] ? (int32_t)std::max(fct_row_blocks(N, M),
                                                                  fct_row_blocks(M, N))
                                              : 0});
    b->part_off[t] = (int32_t)part;
    part += need;
    st_start[t + 1] = st_start[t] + nblk;
  }
  b->st_total = st_start[nt];
  return part;
}

irlsu_status check_ws(const irlsu_plan* pl, const void* ws, size_t bytes) {
  if (!ws || bytes < pl->ws_bytes) return IRLSU_ERR_WORKSPACE;
  return IRLSU_OK;
}

}  // namespace

// ---- augmented form (Algorithm 1 in (U, V^v, V^h)) --------------------------
// Workspace: the plan's layout (setup outputs, preconditioner buffers,
// partial sums, scalars, flags) followed by 16 vectors: x (3), the slack
// blocks of r, z, p, q, b (the U blocks reuse r, z, p0, q, b of the layout)
// and the guard's candidate (3).
static constexpr int kAugExtra = 16;

static size_t aug_bytes(const irlsu_plan* p) {
  const size_t vec = align_up((size_t)p->Np * (size_t)p->Mp * p->elem);
  return layout(p).total + kAugExtra * vec;
}

template <class T>
irlsu_status aug_unwrap_impl(irlsu_plan* pl, const T* X, int64_t ldx, const T* w, const T* Cv,
                             int64_t ldcv, const T* Ch, int64_t ldch, const irlsu_params& prm,
                             double tau, double delta, T* Uout, int64_t ldu, void* ws,
                             irlsu_stats* stats, hipStream_t s) {
  const Ws<T> W = carve<T>(pl, ws);
  const int64_t N = pl->N, M = pl->M, Np = pl->Np, ld = pl->Mp;
  const size_t npx = (size_t)Np * (size_t)ld;
  const size_t vec = align_up(npx * pl->elem);
  char* extra = static_cast<char*>(ws) + layout(pl).total;
  T* ev[kAugExtra];
  for (int i = 0; i < kAugExtra; ++i) ev[i] = reinterpret_cast<T*>(extra + i * vec);
  DevState st = W.st;
  HIP_OK(hipMemsetAsync(st.fl, 0, FL_COUNT * sizeof(int32_t), s));
  HIP_OK(hipMemsetAsync(st.sc, 0, SC_COUNT * sizeof(double), s));
  for (int v = 0; v < V_COUNT; ++v) HIP_OK(hipMemsetAsync(W.v[v], 0, npx * sizeof(T), s));
  for (int i = 0; i < kAugExtra; ++i) HIP_OK(hipMemsetAsync(ev[i], 0, npx * sizeof(T), s));

  SetupArgs<T> sa;
  sa.X = X;
  sa.ldx = ldx;
  sa.w = w;
  sa.Cv = Cv;
  sa.ldcv = ldcv;
  sa.Ch = Ch;
  sa.ldch = ldch;
  sa.U0 = nullptr;
  sa.ldu0 = 0;
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

  AugArgs<T> a;
  a.N = N;
  a.M = M;
  a.Np = Np;
  a.ld = ld;
  a.tau = tau;
  a.delta = delta;
  a.Gv = W.v[V_GV];
  a.Gh = W.v[V_GH];
  a.Cv = W.v[V_CV];
  a.Ch = W.v[V_CH];
  a.dv = W.v[V_OV];
  a.dh = W.v[V_OH];
  a.st = st;
  const AugVec<T> x{ev[0], ev[1], ev[2]};
  const AugVec<T> r{W.v[V_R], ev[3], ev[4]};
  const AugVec<T> z{W.v[V_Z], ev[5], ev[6]};
  const AugVec<T> p{W.v[V_P0], ev[7], ev[8]};
  const AugVec<T> q{W.v[V_Q], ev[9], ev[10]};
  const AugVec<T> b{W.v[V_B], ev[11], ev[12]};
  const AugVec<T> cand{ev[13], ev[14], ev[15]};
  const AugVec<T> none{nullptr, nullptr, nullptr};
  const int guard = prm.sd_guard;
  if (guard != IRLSU_GUARD_OFF)  // 1 / L of Theorem 3 into SC_INVL
    aug_launch<T>(AUG_INVL, a, none, none, none, none, 0, 0, 0, 0.0, s);
  const double tol2 = prm.pcg_rtol * prm.pcg_rtol;
  // right-hand side (fixed by G) and the start U^0 = 0, V^0 = -G
  aug_launch<T>(AUG_RHS, a, x, b, none, none, 1, 0, 0, tol2, s);

  int pcg_total = 0, done_iters = 0;
  irlsu_status overall = IRLSU_OK;
  bool target_hit = false;
  for (int k = 0; k < prm.irls_iters; ++k) {
    aug_launch<T>(AUG_WEIGHTS, a, x, none, none, none, 0, 0, 0, 0.0, s);
    rs = read_back(pl, W, s);
    if (rs != IRLSU_OK) return rs;
    if (stats && k < IRLSU_MAX_IRLS) {
      stats->iter[k].L1 = pl->h_sc[SC_L1];
      stats->iter[k].H = pl->h_sc[SC_H];
      stats->iter[k].pcg_cap = prm.pcg_max;
    }
    if (prm.l1_target > 0.0 && pl->h_sc[SC_L1] <= prm.l1_target) {
      target_hit = true;
      break;
    }
    if (guard != IRLSU_GUARD_OFF) {
      aug_launch<T>(AUG_CAND, a, x, cand, none, none, 0, 0, 0, 0.0, s);
      if (guard == IRLSU_GUARD_CHECK)
        aug_launch<T>(AUG_HVAL, a, cand, none, none, none, SC_SOLD, 0, 0, 0.0, s);
    }
    if (guard == IRLSU_GUARD_CANDIDATE_ONLY) {
      // the remark after Theorem 3: the candidate step replaces the solve
      aug_launch<T>(AUG_GUARD, a, x, cand, none, none, IRLSU_GUARD_CANDIDATE_ONLY, 0, 0, 0.0,
                    s);
      if (stats && k < IRLSU_MAX_IRLS) {
        stats->iter[k].pcg_iters = 0;
        stats->iter[k].status = IRLSU_OK;
        stats->iter[k].relres = 0.0;
        stats->iter[k].guard = 2;
      }
      done_iters = k + 1;
      aug_launch<T>(AUG_CENTER, a, x, none, none, none, 0, 0, 0, 0.0, s);
      continue;
    }
    // ---- Algorithm 2 on the augmented system, warm start from (U, V) ----
    aug_launch<T>(AUG_START, a, none, none, none, none, 0, 0, 0, tol2, s);
    const int nvec = aug_launch<T>(AUG_RESID, a, x, b, r, none, 0, 0, 0, 0.0, s);
    PrecondArgs pa = precond_args<T>(pl, W, r.u, z.u, nullptr, 1, nvec);
    int nzu = launch_precond(pa, s);
    int nzv = aug_launch<T>(AUG_VPRECOND, a, r, z, none, none, 0, 0, 0, 0.0, s);
    for (int l = 0; l < prm.pcg_max; ++l) {
      aug_launch<T>(AUG_PUPDATE, a, z, p, none, none, l, nzu, nzv, 0.0, s);
      const int npq = aug_launch<T>(AUG_APPLY, a, p, q, none, none, 0, 0, 0, 0.0, s);
      aug_launch<T>(AUG_AXPY, a, x, r, p, q, l, npq, 0, 0.0, s);
      if (prm.true_res_every > 0 && (l + 1) % prm.true_res_every == 0 && l + 1 < prm.pcg_max)
        aug_launch<T>(AUG_RESID, a, x, b, r, none, 1, 0, 0, 0.0, s);
      if (l + 1 < prm.pcg_max) {
        nzu = launch_precond(pa, s);
        nzv = aug_launch<T>(AUG_VPRECOND, a, r, z, none, none, 0, 0, 0, 0.0, s);
      }
      if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
      if (prm.poll_every > 0 && (l + 1) % prm.poll_every == 0) {
        HIP_OK(hipMemcpyAsync(pl->h_flags, st.fl, FL_COUNT * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (pl->h_flags[FL_DONE]) break;
      }
    }
    launch_finalize_rr(st, nvec, s);
    if (guard == IRLSU_GUARD_CHECK) {
      aug_launch<T>(AUG_HVAL, a, x, none, none, none, SC_SNEW, 0, 0, 0.0, s);
      aug_launch<T>(AUG_GUARD, a, x, cand, none, none, IRLSU_GUARD_CHECK, 0, 0, 0.0, s);
    }
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
      stats->iter[k].guard = guard == IRLSU_GUARD_CHECK ? pl->h_flags[FL_GUARD] : 0;
    }
    pcg_total += iters;
    done_iters = k + 1;
    if (solve_st == IRLSU_ERR_BREAKDOWN) return IRLSU_ERR_BREAKDOWN;
    if (solve_st == IRLSU_NOT_CONVERGED) overall = IRLSU_NOT_CONVERGED;
    aug_launch<T>(AUG_CENTER, a, x, none, none, none, 0, 0, 0, 0.0, s);
  }
  aug_launch<T>(AUG_WEIGHTS, a, x, none, none, none, 0, 0, 0, 0.0, s);
  rs = read_back(pl, W, s);
  if (rs != IRLSU_OK) return rs;
  if (prm.l1_target > 0.0 && pl->h_sc[SC_L1] <= prm.l1_target) target_hit = true;
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
  HIP_OK(hipMemcpy2DAsync(Uout, (size_t)ldu * sizeof(T), x.u, (size_t)ld * sizeof(T),
                          (size_t)M * sizeof(T), (size_t)N, hipMemcpyDeviceToDevice, s));
  if (stats) HIP_OK(hipStreamSynchronize(s));
  return overall;
}

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
  p->cg_schedule = IRLSU_CG_FIXED;
  p->cg_m0 = 5;
  p->cg_eps_tol = 1e-3;
  p->cg_alpha = 1.7;
  p->sd_guard = IRLSU_GUARD_CHECK;
  p->graph = 1;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_create(irlsu_plan** out, int64_t N, int64_t M, irlsu_precision prec,
                               void* stream) {
  return irlsu_plan_create_ex(out, N, M, prec, IRLSU_PLAN_AUTO, stream);
}

irlsu_status irlsu_plan_create_ex(irlsu_plan** out, int64_t N, int64_t M, irlsu_precision prec,
                                  int32_t form, void* stream) {
  if (!out) return IRLSU_ERR_INVALID_ARG;
  *out = nullptr;
  if (N < 2 || M < 2) return IRLSU_ERR_SHAPE;
  if (prec < IRLSU_F64 || prec > IRLSU_MIXED_F16) return IRLSU_ERR_UNSUPPORTED;
  if (form < IRLSU_PLAN_AUTO || form > IRLSU_PLAN_FAST) return IRLSU_ERR_INVALID_ARG;
  if (N > kMaxSide || M > kMaxSide) return IRLSU_ERR_SHAPE;
  const bool even = (N % 2 == 0) && (M % 2 == 0);
  if (form == IRLSU_PLAN_FOLDED && !even) return IRLSU_ERR_SHAPE;
  const bool pow2 = fct_supported(N) && fct_supported(M);
  // sides with factors 2, 3 and 5 only (a multiple of 8, half at most 8192)
  const bool general = !pow2 && fctg_supported(N) && fctg_supported(M);
  if (form == IRLSU_PLAN_FAST && !pow2 && !general) return IRLSU_ERR_SHAPE;
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
  // the fast form wherever it applies; else the folded form once the
  // products dominate its extra passes
  p->fast = form == IRLSU_PLAN_FAST || (form == IRLSU_PLAN_AUTO && (pow2 || general));
  p->folded = !p->fast && (form == IRLSU_PLAN_FOLDED ||
                           (form == IRLSU_PLAN_AUTO && even && p->Np * p->Mp >= ((int64_t)1 << 20)));
  p->hNp = round_up(N / 2, kTilePad);
  p->hMp = round_up(M / 2, kTilePad);
  // the GEMM grids and the partial-sum table bound the supported size
  const int64_t tiles = (p->Np / 64) * (p->Mp / 64);
  if (tiles > kMaxPartials) {
    delete p;
    return IRLSU_ERR_SHAPE;
  }
  (void)hipGetDevice(&p->device);
  // set-up of irlsu_operator_noalloc on this device (its scratch address);
  // a failure here surfaces as ERR_HIP from that entry point
  (void)scratch_address(p->device);
  bool ok = true;
  if (p->fast) {
    const bool share = (N == M);
    const size_t bN = fct_table_bytes(N, p->elem), bM = fct_table_bytes(M, p->elem);
    ok = dev_malloc(&p->twN, bN) == hipSuccess &&
         dev_malloc(reinterpret_cast<void**>(&p->eigN), N * sizeof(double)) == hipSuccess;
    if (ok && !share)
      ok = dev_malloc(&p->twM, bM) == hipSuccess &&
           dev_malloc(reinterpret_cast<void**>(&p->eigM), M * sizeof(double)) == hipSuccess;
    if (ok && share) {
      p->twM = p->twN;
      p->eigM = p->eigN;
    }
    p->plan_bytes = bN + N * sizeof(double) + (share ? 0 : bM + M * sizeof(double));
  } else if (p->folded) {
    const bool share = (N == M);
    const size_t bN = (size_t)p->hNp * p->hNp * p->opsz;
    const size_t bM = (size_t)p->hMp * p->hMp * p->opsz;
    ok = dev_malloc(&p->PeN, bN) == hipSuccess && dev_malloc(&p->PeNt, bN) == hipSuccess &&
         dev_malloc(&p->PoN, bN) == hipSuccess && dev_malloc(&p->PoNt, bN) == hipSuccess &&
         dev_malloc(reinterpret_cast<void**>(&p->eigNf), 2 * p->hNp * sizeof(double)) == hipSuccess;
    if (ok && !share) {
      ok = dev_malloc(&p->PeM, bM) == hipSuccess && dev_malloc(&p->PeMt, bM) == hipSuccess &&
           dev_malloc(&p->PoM, bM) == hipSuccess && dev_malloc(&p->PoMt, bM) == hipSuccess &&
           dev_malloc(reinterpret_cast<void**>(&p->eigMf), 2 * p->hMp * sizeof(double)) == hipSuccess;
    }
    if (ok && share) {
      p->PeM = p->PeN;
      p->PeMt = p->PeNt;
      p->PoM = p->PoN;
      p->PoMt = p->PoNt;
      p->eigMf = p->eigNf;
    }
    p->plan_bytes = 4 * bN + 2 * p->hNp * sizeof(double) +
                    (share ? 0 : 4 * bM + 2 * p->hMp * sizeof(double));
  } else {
    const bool share = (p->Np == p->Mp) && (N == M);
    const size_t bN = (size_t)p->Np * p->Np * p->opsz;
    const size_t bM = (size_t)p->Mp * p->Mp * p->opsz;
    ok = dev_malloc(&p->PN, bN) == hipSuccess && dev_malloc(&p->PNt, bN) == hipSuccess &&
         dev_malloc(reinterpret_cast<void**>(&p->eigN), p->Np * sizeof(double)) == hipSuccess;
    if (ok && !share) {
      ok = dev_malloc(&p->PM, bM) == hipSuccess && dev_malloc(&p->PMt, bM) == hipSuccess &&
           dev_malloc(reinterpret_cast<void**>(&p->eigM), p->Mp * sizeof(double)) == hipSuccess;
    }
    if (ok && share) {
      p->PM = p->PN;
      p->PMt = p->PNt;
      p->eigM = p->eigN;
    }
    p->plan_bytes = 2 * bN + p->Np * sizeof(double) + (share ? 0 : 2 * bM + p->Mp * sizeof(double));
  }
  ok = ok && pinned_malloc(reinterpret_cast<void**>(&p->h_flags), 256, hipHostMallocDefault) == hipSuccess;
  ok = ok && pinned_malloc(reinterpret_cast<void**>(&p->h_sc), 512, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    irlsu_plan_destroy(p);
    return IRLSU_ERR_OOM;
  }
  if (p->fast) {
    launch_fct_tables(p->elem, N, p->twN, p->eigN, s, general);
    if (p->twM != p->twN) launch_fct_tables(p->elem, M, p->twM, p->eigM, s, general);
  } else if (p->folded) {
    launch_fold_basis(p->kind, N, p->hNp, p->PeN, p->PeNt, p->PoN, p->PoNt, p->eigNf, s);
    if (p->PeM != p->PeN)
      launch_fold_basis(p->kind, M, p->hMp, p->PeM, p->PeMt, p->PoM, p->PoMt, p->eigMf, s);
  } else {
    launch_basis(p->kind, N, p->Np, p->PN, p->PNt, p->eigN, s);
    if (p->PM != p->PN) launch_basis(p->kind, M, p->Mp, p->PM, p->PMt, p->eigM, s);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    irlsu_plan_destroy(p);
    return IRLSU_ERR_HIP;
  }
  p->ws_bytes = layout(p).total;
  // the capture stream of the PCG graphs; without it the loop launches
  // directly (irlsu_params.graph is then ignored)
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    p->cap_stream = nullptr;
  }
  for (hipEvent_t& e : p->poll_ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
    }
  }
  *out = p;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_destroy(irlsu_plan* p) {
  if (!p) return IRLSU_OK;
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->poll_ev)
    if (e) (void)hipEventDestroy(e);
  if (p->prof) {
    for (int i = 0; i <= LaunchLog::kMax; ++i) (void)hipEventDestroy(p->prof->ev[i]);
    delete p->prof;
  }
  const bool fshare = p->PeM == p->PeN;
  void* fold_n[] = {p->PeN, p->PeNt, p->PoN, p->PoNt, p->eigNf};
  void* fold_m[] = {p->PeM, p->PeMt, p->PoM, p->PoMt, p->eigMf};
  for (void* q : fold_n) if (q) (void)hipFree(q);
  if (!fshare) for (void* q : fold_m) if (q) (void)hipFree(q);
  if (p->twN) (void)hipFree(p->twN);
  if (p->twM && p->twM != p->twN) (void)hipFree(p->twM);
  const bool share = p->PM == p->PN;
  if (p->PN) (void)hipFree(p->PN);
  if (p->PNt) (void)hipFree(p->PNt);
  if (!share) {
    if (p->PM) (void)hipFree(p->PM);
    if (p->PMt) (void)hipFree(p->PMt);
  }
  if (p->eigN) (void)hipFree(p->eigN);
  if (p->eigM && p->eigM != p->eigN) (void)hipFree(p->eigM);
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
  out->folded = p->folded;
  out->form = p->fast ? IRLSU_PLAN_FAST : (p->folded ? IRLSU_PLAN_FOLDED : IRLSU_PLAN_DENSE);
  return IRLSU_OK;
}

size_t irlsu_workspace_bytes(const irlsu_plan* p) { return p ? p->ws_bytes : 0; }

void irlsu_test_fail_alloc(int32_t nth) { g_fail_alloc_at = nth < 0 ? -1 : nth; }

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
  if (prm.cg_schedule != IRLSU_CG_FIXED &&
      (prm.cg_schedule != IRLSU_CG_ADAPTIVE || prm.cg_m0 < 1 || !(prm.cg_alpha >= 1.0) ||
       !(prm.cg_eps_tol >= 0.0)))
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

static irlsu_status adjoint_entry(irlsu_plan* plan, const void* gU, int64_t ldg,
                                  const irlsu_params* params, void* gCv, int64_t ldgcv, void* gCh,
                                  int64_t ldgch, void* gX, int64_t ldgx, void* workspace,
                                  size_t workspace_bytes, irlsu_stats* stats, void* stream,
                                  bool implicit) {
  if (!plan || !gU || !gCv || !gCh) return IRLSU_ERR_INVALID_ARG;
  if (ldg < plan->M || ldgcv < plan->M || ldgch < plan->M - 1) return IRLSU_ERR_INVALID_ARG;
  if (gX && ldgx < plan->M) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  irlsu_params prm;
  if (params) prm = *params;
  else irlsu_params_default(&prm, plan->prec);
  if (!(prm.eps > 0.0) || prm.pcg_max < 1 || prm.poll_every < 0 || prm.true_res_every < 0)
    return IRLSU_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->elem == 8)
    return adjoint_impl<double>(plan, static_cast<const double*>(gU), ldg, prm,
                                static_cast<double*>(gCv), ldgcv, static_cast<double*>(gCh), ldgch,
                                static_cast<double*>(gX), ldgx, workspace, stats, s, implicit);
  return adjoint_impl<float>(plan, static_cast<const float*>(gU), ldg, prm,
                             static_cast<float*>(gCv), ldgcv, static_cast<float*>(gCh), ldgch,
                             static_cast<float*>(gX), ldgx, workspace, stats, s, implicit);
}

irlsu_status irlsu_adjoint(irlsu_plan* plan, const void* gU, int64_t ldg,
                           const irlsu_params* params, void* gCv, int64_t ldgcv, void* gCh,
                           int64_t ldgch, void* gX, int64_t ldgx, void* workspace,
                           size_t workspace_bytes, irlsu_stats* stats, void* stream) {
  return adjoint_entry(plan, gU, ldg, params, gCv, ldgcv, gCh, ldgch, gX, ldgx, workspace,
                       workspace_bytes, stats, stream, false);
}

irlsu_status irlsu_adjoint_implicit(irlsu_plan* plan, const void* gU, int64_t ldg,
                                    const irlsu_params* params, void* gCv, int64_t ldgcv,
                                    void* gCh, int64_t ldgch, void* gX, int64_t ldgx,
                                    void* workspace, size_t workspace_bytes, irlsu_stats* stats,
                                    void* stream) {
  return adjoint_entry(plan, gU, ldg, params, gCv, ldgcv, gCh, ldgch, gX, ldgx, workspace,
                       workspace_bytes, stats, stream, true);
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

irlsu_status irlsu_operator_noalloc(const irlsu_plan* plan, const void* Ov, const void* Oh,
                                    const void* p, void* q, double* pq, void* stream) {
  if (!plan || !Ov || !Oh || !p || !q) return IRLSU_ERR_INVALID_ARG;
  if (p == q) return IRLSU_ERR_INVALID_ARG;
  int rows = 0;
  const dim3 g = stencil_grid(plan->Np, plan->Mp, &rows, plan->tune_rows);
  if ((int64_t)g.x * (int64_t)g.y > kNoAllocParts) return IRLSU_ERR_SHAPE;
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != plan->device) return IRLSU_ERR_INVALID_ARG;
  double* sp = scratch_address(dev);
  if (!sp) return IRLSU_ERR_HIP;
  DevState st;
  st.part = sp;
  st.off = 0;
  st.stride = kNoAllocParts;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) {
    using T = decltype(tag);
    StencilArgs<T> a = stencil_base<T>(plan, static_cast<const T*>(Ov), static_cast<const T*>(Oh),
                                       st);
    a.p_in = static_cast<const T*>(p);
    a.q = static_cast<T*>(q);
    a.check_done = 0;
    const int n = launch_stencil<T>(ST_APPLY, a, s);
    if (pq) launch_reduce_to(st, PR_PQ, n, pq, s);
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
    int nrr = 0;
    if constexpr (sizeof(T) == 4) {
      if (plan->kind == OK_F16)
        nrr = launch_sumsq<float>(static_cast<const float*>(r), plan->Np * plan->Mp, W.st, s);
    }
    PrecondArgs a = precond_args<T>(plan, W, static_cast<const T*>(r), static_cast<T*>(z), nullptr,
                                    0, nrr);
    const int n = launch_precond(a, s);
    if (rz) launch_reduce_to(W.st, PR_ZR, n, rz, s);
    return IRLSU_OK;
  };
  st = plan->elem == 8 ? go(double{}) : go(float{});
  if (st != IRLSU_OK) return st;
  return last_launch();
}

irlsu_status irlsu_pcg(irlsu_plan* plan, const void* Ov, const void* Oh, const void* b, double* x,
                       const irlsu_params* params, int32_t* iters, double* relres,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !Ov || !Oh || !b || !x) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  irlsu_params prm;
  if (params) {
    prm = *params;
  } else {
    irlsu_params_default(&prm, plan->prec);
  }
  if (!(prm.pcg_rtol >= 0.0) || prm.pcg_max < 1 || prm.true_res_every < 0 || prm.poll_every < 0)
    return IRLSU_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t npx = (size_t)plan->Np * (size_t)plan->Mp;
  int it = 0;
  double rel = 0.0;
  irlsu_status solve_st = IRLSU_OK;
  auto go = [&](auto tag) -> irlsu_status {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    // the weights where the loop's kernels read them; the right-hand side
    // projected on the range of the operator (mean zero), with ||b||^2, the
    // tolerance and cleared flags for the solve
    HIP_OK(hipMemcpyAsync(W.v[V_OV], Ov, npx * sizeof(T), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(W.v[V_OH], Oh, npx * sizeof(T), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemsetAsync(W.st.sc, 0, SC_COUNT * sizeof(double), s));
    // the loop's vectors start from zero: the first direction update
    // multiplies the previous direction by beta = 0, which keeps stale
    // non-finite workspace contents from entering
    for (int v : {V_R, V_Z, V_P0, V_P1, V_Q, V_D})
      HIP_OK(hipMemsetAsync(W.v[v], 0, npx * sizeof(T), s));
    launch_adjoint_rhs<T>(static_cast<const T*>(b), plan->Mp, plan->N, plan->M, plan->Np,
                          plan->Mp, W.v[V_B], W.st, prm.pcg_rtol * prm.pcg_rtol, s);
    if (last_launch() != IRLSU_OK) return IRLSU_ERR_HIP;
    const int flexible = prm.flexible < 0 ? default_flexible(plan) : prm.flexible;
    return pcg_solve<T>(plan, W, x, W.v[V_B], prm, flexible, &it, &rel, &solve_st, s);
  };
  st = plan->elem == 8 ? go(double{}) : go(float{});
  if (st != IRLSU_OK) return st;
  if (iters) *iters = it;
  if (relres) *relres = rel;
  return solve_st;
}

irlsu_status irlsu_stream_probe(int32_t kind, const void* a, const void* b, const void* c, void* d,
                                size_t bytes, int32_t grid, int32_t reps, double* ms,
                                void* stream) {
  if (kind < IRLSU_PROBE_COPY || kind > IRLSU_PROBE_3R1W || !a || !ms || grid < 1 || reps < 1 ||
      bytes < 16 || bytes % 16 != 0)
    return IRLSU_ERR_INVALID_ARG;
  if (kind != IRLSU_PROBE_READ && !d) return IRLSU_ERR_INVALID_ARG;
  if (kind == IRLSU_PROBE_3R1W && (!b || !c)) return IRLSU_ERR_INVALID_ARG;
  float t = 0.f;
  if (launch_stream_probe(kind, a, b, c, d, bytes, grid, reps, &t,
                          static_cast<hipStream_t>(stream)) != 0)
    return IRLSU_ERR_HIP;
  *ms = (double)t;
  return IRLSU_OK;
}

irlsu_status irlsu_precond_timed(const irlsu_plan* plan, const void* r, void* z, void* workspace,
                                 size_t workspace_bytes, int32_t reps, double* ms_launch,
                                 int32_t* kind, int32_t* n_launches, void* stream) {
  if (!plan || !r || !z || r == z || reps < 1 || !ms_launch || !kind || !n_launches)
    return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LaunchLog L;
  int created = 0;
  for (; created <= LaunchLog::kMax; ++created)
    if (hipEventCreate(&L.ev[created]) != hipSuccess) break;
  auto destroy = [&]() {
    for (int i = 0; i < created; ++i) (void)hipEventDestroy(L.ev[i]);
  };
  if (created <= LaunchLog::kMax) {
    destroy();
    return IRLSU_ERR_HIP;
  }
  for (int i = 0; i < LaunchLog::kMax; ++i) {
    ms_launch[i] = 0.0;
    kind[i] = -1;
  }
  *n_launches = 0;
  auto go = [&](auto tag) -> irlsu_status {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    for (int rep = 0; rep < reps; ++rep) {
      HIP_OK(hipMemsetAsync(W.st.fl, 0, FL_COUNT * sizeof(int32_t), s));
      int nrr = 0;
      if constexpr (sizeof(T) == 4) {
        if (plan->kind == OK_F16)
          nrr = launch_sumsq<float>(static_cast<const float*>(r), plan->Np * plan->Mp, W.st, s);
      }
      PrecondArgs a = precond_args<T>(plan, W, static_cast<const T*>(r), static_cast<T*>(z),
                                      nullptr, 0, nrr);
      a.log = &L;
      L.n = 0;
      launch_precond(a, s);
      HIP_OK(hipEventSynchronize(L.ev[L.n]));
      *n_launches = L.n;
      for (int i = 0; i < L.n; ++i) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, L.ev[i], L.ev[i + 1]));
        ms_launch[i] += ms / reps;
        kind[i] = L.cls[i];
      }
    }
    return IRLSU_OK;
  };
  st = plan->elem == 8 ? go(double{}) : go(float{});
  destroy();
  if (st != IRLSU_OK) return st;
  return last_launch();
}

irlsu_status irlsu_profile_arm(irlsu_plan* plan, int32_t irls_k, int32_t pcg_l) {
  if (!plan) return IRLSU_ERR_INVALID_ARG;
  plan->prof_k = irls_k;
  plan->prof_l = pcg_l;
  if (irls_k < 0 || pcg_l < 0) {
    plan->prof_k = plan->prof_l = -1;
    return IRLSU_OK;
  }
  if (!plan->prof) {
    LaunchLog* L = new (std::nothrow) LaunchLog;
    if (!L) return IRLSU_ERR_OOM;
    int created = 0;
    for (; created <= LaunchLog::kMax; ++created)
      if (hipEventCreate(&L->ev[created]) != hipSuccess) break;
    if (created <= LaunchLog::kMax) {
      for (int i = 0; i < created; ++i) (void)hipEventDestroy(L->ev[i]);
      delete L;
      return IRLSU_ERR_HIP;
    }
    plan->prof = L;
  }
  plan->prof->n = 0;
  return IRLSU_OK;
}

irlsu_status irlsu_profile_result(irlsu_plan* plan, double* ms_launch, int32_t* kind,
                                  int32_t* n_launches) {
  if (!plan || !ms_launch || !kind || !n_launches) return IRLSU_ERR_INVALID_ARG;
  *n_launches = 0;
  LaunchLog* L = plan->prof;
  if (!L || L->n == 0) return IRLSU_OK;
  HIP_OK(hipEventSynchronize(L->ev[L->n]));
  for (int i = 0; i < L->n; ++i) {
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, L->ev[i], L->ev[i + 1]));
    ms_launch[i] = ms;
    kind[i] = L->cls[i];
  }
  *n_launches = L->n;
  return IRLSU_OK;
}

irlsu_status irlsu_round_congruent(const irlsu_plan* plan, const void* X, int64_t ldx,
                                   const void* U, int64_t ldu, void* out, int64_t ldo,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !X || !U || !out || ldx < plan->M || ldu < plan->M || ldo < plan->M)
    return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->elem == 8) {
    const Ws<double> W = carve<double>(plan, workspace);
    launch_congruent<double>(static_cast<const double*>(X), ldx, static_cast<const double*>(U),
                             ldu, static_cast<double*>(out), ldo, plan->N, plan->M, W.st, s);
  } else {
    const Ws<float> W = carve<float>(plan, workspace);
    launch_congruent<float>(static_cast<const float*>(X), ldx, static_cast<const float*>(U), ldu,
                            static_cast<float*>(out), ldo, plan->N, plan->M, W.st, s);
  }
  return last_launch();
}

size_t irlsu_augmented_workspace_bytes(const irlsu_plan* plan) {
  return plan ? aug_bytes(plan) : 0;
}

irlsu_status irlsu_unwrap_augmented(irlsu_plan* plan, const void* X, int64_t ldx, const void* w,
                                    const void* Cv, int64_t ldcv, const void* Ch, int64_t ldch,
                                    const irlsu_params* params, double tau, double delta,
                                    void* U, int64_t ldu, void* workspace,
                                    size_t workspace_bytes, irlsu_stats* stats, void* stream) {
  if (!plan || !X || !U || !workspace || ldx < plan->M || ldu < plan->M) return IRLSU_ERR_INVALID_ARG;
  if ((Cv == nullptr) != (Ch == nullptr)) return IRLSU_ERR_INVALID_ARG;
  if (Cv && (ldcv < plan->M || ldch < plan->M - 1)) return IRLSU_ERR_INVALID_ARG;
  if (!(tau > 0.0) || !(delta > 0.0)) return IRLSU_ERR_INVALID_ARG;
  if (workspace_bytes < aug_bytes(plan)) return IRLSU_ERR_WORKSPACE;
  irlsu_params prm;
  if (params) {
    prm = *params;
  } else {
    irlsu_params_default(&prm, plan->prec);
  }
  if (prm.irls_iters < 0 || prm.pcg_max < 1 || prm.true_res_every < 0 || prm.poll_every < 0 ||
      !(prm.pcg_rtol >= 0.0) || prm.sd_guard < IRLSU_GUARD_OFF ||
      prm.sd_guard > IRLSU_GUARD_CANDIDATE_ONLY)
    return IRLSU_ERR_INVALID_ARG;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->elem == 8)
    return aug_unwrap_impl<double>(plan, static_cast<const double*>(X), ldx,
                                   static_cast<const double*>(w), static_cast<const double*>(Cv),
                                   ldcv, static_cast<const double*>(Ch), ldch, prm, tau, delta,
                                   static_cast<double*>(U), ldu, workspace, stats, s);
  return aug_unwrap_impl<float>(plan, static_cast<const float*>(X), ldx,
                                static_cast<const float*>(w), static_cast<const float*>(Cv), ldcv,
                                static_cast<const float*>(Ch), ldch, prm, tau, delta,
                                static_cast<float*>(U), ldu, workspace, stats, s);
}

irlsu_status irlsu_batch_destroy(irlsu_batch* b) {
  if (!b) return IRLSU_OK;
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (hipEvent_t e : b->poll_ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : b->P) if (p) (void)hipFree(p);
  for (void* p : b->Pt) if (p) (void)hipFree(p);
  for (double* p : b->eig) if (p) (void)hipFree(p);
  for (void* p : b->tw) if (p) (void)hipFree(p);
  for (double* p : b->eigf) if (p) (void)hipFree(p);
  if (b->d_st_start) (void)hipFree(b->d_st_start);
  if (b->d_g_start) (void)hipFree(b->d_g_start);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->h_tiles) (void)hipHostFree(b->h_tiles);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  if (b->h_sc) (void)hipHostFree(b->h_sc);
  delete b;
  return IRLSU_OK;
}

irlsu_status irlsu_batch_create(irlsu_batch** out, const int64_t* shapes, int32_t ntiles,
                                irlsu_precision prec, void* stream) {
  if (!out || !shapes || ntiles < 1) return IRLSU_ERR_INVALID_ARG;
  *out = nullptr;
  if (prec != IRLSU_MIXED_BF16 && prec != IRLSU_MIXED_F16 && prec != IRLSU_F32)
    return IRLSU_ERR_UNSUPPORTED;
  for (int t = 0; t < ntiles; ++t)
    if (shapes[2 * t] < 2 || shapes[2 * t + 1] < 2 || shapes[2 * t] > kMaxSide ||
        shapes[2 * t + 1] > kMaxSide)
      return IRLSU_ERR_SHAPE;
  irlsu_batch* b = new (std::nothrow) irlsu_batch;
  if (!b) return IRLSU_ERR_OOM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  b->ntiles = ntiles;
  b->prec = prec;
  b->kind = prec == IRLSU_MIXED_F16 ? OK_F16 : (prec == IRLSU_F32 ? OK_F32 : OK_BF16);
  b->opsz = prec == IRLSU_F32 ? 4 : 2;
  std::vector<int32_t> st_start, g_start(4 * (ntiles + 1), 0);
  size_t off = 0;
  for (int t = 0; t < ntiles; ++t) {
    const int64_t N = shapes[2 * t], M = shapes[2 * t + 1];
    const int64_t Np = round_up(N, kBatchPad), Mp = round_up(M, kBatchPad);
    b->N.push_back(N);
    b->M.push_back(M);
    b->Np.push_back(Np);
    b->Mp.push_back(Mp);
    int gb[4];
    const bool fast = batch_tile_fast(N, M);
    b->fast.push_back(fast ? 1 : 0);
    if (fast) {
      gb[0] = gb[1] = gb[2] = gb[3] = 0;  // no grouped products: its own passes
    } else {
      precond_blocks(b->kind, Np, Mp, gb);
    }
    for (int q = 0; q < 4; ++q) g_start[q * (ntiles + 1) + t + 1] = g_start[q * (ntiles + 1) + t] + gb[q];
    b->tile_off.push_back(off);
    off += align_up(batch_tile_bytes(Np, Mp, b->opsz));
    if (fast) {
      b->fast_side_index.emplace(N, 0);
      b->fast_side_index.emplace(M, 0);
    } else {
      b->side_index.emplace(N, 0);
      b->side_index.emplace(M, 0);
    }
  }
  if (batch_grids(b, std::vector<int>(ntiles, 0), st_start) > kMaxPartials) {
    irlsu_batch_destroy(b);
    return IRLSU_ERR_SHAPE;
  }
  for (int q = 0; q < 4; ++q) b->g_total[q] = g_start[q * (ntiles + 1) + ntiles];
  b->part_off_bytes = off;
  off = align_up(off + (size_t)kPartSlots * kMaxPartials * sizeof(double));
  b->sc_off = off;
  off = align_up(off + (size_t)ntiles * SC_COUNT * sizeof(double));
  b->fl_off = off;
  off = align_up(off + (size_t)ntiles * FL_COUNT * sizeof(int32_t));
  b->ws_bytes = off;
  bool ok = true;
  int idx = 0;
  for (auto& kv : b->side_index) {
    kv.second = idx++;
    const int64_t n = kv.first, npad = round_up(n, kBatchPad);
    void *P = nullptr, *Pt = nullptr;
    double* e = nullptr;
    ok = ok && dev_malloc(&P, (size_t)npad * npad * b->opsz) == hipSuccess;
    ok = ok && dev_malloc(&Pt, (size_t)npad * npad * b->opsz) == hipSuccess;
    ok = ok && dev_malloc(reinterpret_cast<void**>(&e), npad * sizeof(double)) == hipSuccess;
    b->P.push_back(P);
    b->Pt.push_back(Pt);
    b->eig.push_back(e);
    if (ok) launch_basis(b->kind, n, npad, P, Pt, e, s);
  }
  idx = 0;
  for (auto& kv : b->fast_side_index) {
    kv.second = idx++;
    const int64_t n = kv.first;
    void* tw = nullptr;
    double* e = nullptr;
    ok = ok && dev_malloc(&tw, fct_table_bytes(n, 4)) == hipSuccess;
    ok = ok && dev_malloc(reinterpret_cast<void**>(&e), n * sizeof(double)) == hipSuccess;
    b->tw.push_back(tw);
    b->eigf.push_back(e);
    if (ok) launch_fct_tables(4, n, tw, e, s);
  }
  ok = ok && dev_malloc(reinterpret_cast<void**>(&b->d_st_start), st_start.size() * 4) == hipSuccess;
  ok = ok && dev_malloc(reinterpret_cast<void**>(&b->d_g_start), g_start.size() * 4) == hipSuccess;
  ok = ok && dev_malloc(&b->d_tiles, (size_t)ntiles * sizeof(BatchTile<float>)) == hipSuccess;
  ok = ok && pinned_malloc(&b->h_tiles, (size_t)ntiles * sizeof(BatchTile<float>),
                           hipHostMallocDefault) == hipSuccess;
  ok = ok && pinned_malloc(reinterpret_cast<void**>(&b->h_flags), (size_t)ntiles * FL_COUNT * 8,
                           hipHostMallocDefault) == hipSuccess;
  ok = ok && pinned_malloc(reinterpret_cast<void**>(&b->h_sc), (size_t)ntiles * SC_COUNT * 8,
                           hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    irlsu_batch_destroy(b);
    return IRLSU_ERR_OOM;
  }
  if (hipMemcpy(b->d_st_start, st_start.data(), st_start.size() * 4, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->d_g_start, g_start.data(), g_start.size() * 4, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    irlsu_batch_destroy(b);
    return IRLSU_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    b->cap_stream = nullptr;
  }
  for (hipEvent_t& e : b->poll_ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
    }
  }
  *out = b;
  return IRLSU_OK;
}

size_t irlsu_batch_workspace_bytes(const irlsu_batch* b) { return b ? b->ws_bytes : 0; }

irlsu_status irlsu_unwrap_batched(irlsu_batch* b, const irlsu_tile* tiles,
                                  const irlsu_params* params, void* workspace,
                                  size_t workspace_bytes, irlsu_stats* stats, void* stream) {
  if (!b || !tiles) return IRLSU_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < b->ws_bytes) return IRLSU_ERR_WORKSPACE;
  for (int t = 0; t < b->ntiles; ++t) {
    const irlsu_tile& x = tiles[t];
    if (!x.X || !x.U || x.ldx < b->M[t] || x.ldu < b->M[t]) return IRLSU_ERR_INVALID_ARG;
    if ((x.Cv == nullptr) != (x.Ch == nullptr)) return IRLSU_ERR_INVALID_ARG;
    if (x.Cv && (x.ldcv < b->M[t] || x.ldch < b->M[t] - 1)) return IRLSU_ERR_INVALID_ARG;
  }
  irlsu_params prm;
  if (params) prm = *params;
  else irlsu_params_default(&prm, b->prec);
  if (!(prm.eps > 0.0) || !(prm.pcg_rtol >= 0.0) || prm.irls_iters < 0 || prm.pcg_max < 1 ||
      prm.true_res_every < 0 || prm.poll_every < 0 || prm.irls_iters >= IRLSU_MAX_IRLS)
    return IRLSU_ERR_INVALID_ARG;
  return unwrap_batched_impl(b, tiles, prm, workspace, stats, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---- autotuner -------------------------------------------------------------
namespace {

int plan_form(const irlsu_plan* p) {
  return p->fast ? IRLSU_PLAN_FAST : (p->folded ? IRLSU_PLAN_FOLDED : IRLSU_PLAN_DENSE);
}

void put_tune(irlsu_tune* out, int rows, int upd, int small, int from_cache, double su, double uu,
              double pu) {
  if (!out) return;
  out->stencil_rows = rows;
  out->update_blocks = upd;
  out->small_tiles = small;
  out->from_cache = from_cache;
  out->stencil_us = su;
  out->update_us = uu;
  out->precond_us = pu;
}

constexpr int kRowCands[] = {8, 16, 32, 64, 128, 256};
constexpr int kUpdateCands[] = {64, 128, 256, 512, 1024, 2048, 4096};

}  // namespace

irlsu_status irlsu_plan_set_tune(irlsu_plan* plan, const irlsu_tune* t) {
  if (!plan) return IRLSU_ERR_INVALID_ARG;
  if (t && (t->stencil_rows < 0 || t->update_blocks < 0 || t->small_tiles < 0 ||
            t->small_tiles > 1))
    return IRLSU_ERR_INVALID_ARG;
  plan->tune_rows = t ? t->stencil_rows : 0;
  plan->tune_update = t ? t->update_blocks : 0;
  plan->tune_small = t ? t->small_tiles : 0;
  return IRLSU_OK;
}

irlsu_status irlsu_plan_get_tune(const irlsu_plan* plan, irlsu_tune* out) {
  if (!plan || !out) return IRLSU_ERR_INVALID_ARG;
  put_tune(out, plan->tune_rows, plan->tune_update, plan->tune_small, 0, 0.0, 0.0, 0.0);
  return IRLSU_OK;
}

irlsu_status irlsu_plan_autotune(irlsu_plan* plan, const char* cache_path, irlsu_tune* out,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return IRLSU_ERR_INVALID_ARG;
  irlsu_status st = check_ws(plan, workspace, workspace_bytes);
  if (st != IRLSU_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  TuneEntry key;
  key.kind = "plan";
  key.arch = device_arch(plan->device);
  key.N = plan->N;
  key.M = plan->M;
  key.precision = plan->prec;
  key.form = plan_form(plan);
  std::vector<TuneEntry> cache = tune_cache_read(cache_path);
  if (const TuneEntry* e = tune_cache_find(cache, key)) {
    plan->tune_rows = e->stencil_rows;
    plan->tune_update = e->update_blocks;
    plan->tune_small = e->small_tiles;
    put_tune(out, e->stencil_rows, e->update_blocks, e->small_tiles, 1, e->stencil_us,
             e->update_us, e->precond_us);
    return IRLSU_OK;
  }
  double su = 0.0, uu = 0.0, pu = 0.0;
  auto go = [&](auto tag) -> irlsu_status {
    using T = decltype(tag);
    const Ws<T> W = carve<T>(plan, workspace);
    const size_t npx = (size_t)plan->Np * (size_t)plan->Mp;
    for (int v : {V_OV, V_OH, V_P0, V_Q, V_R, V_Z, V_D})
      HIP_OK(hipMemsetAsync(W.v[v], 0, npx * sizeof(T), s));
    HIP_OK(hipMemsetAsync(W.U, 0, npx * sizeof(double), s));
    HIP_OK(hipMemsetAsync(W.st.sc, 0, SC_COUNT * sizeof(double), s));
    HIP_OK(hipMemsetAsync(W.st.fl, 0, FL_COUNT * sizeof(int32_t), s));
    // 1) band height of the operator (its plain apply form)
    int best_rows = 0;
    double best = 0.0;
    for (int cand = -1; cand < (int)(sizeof(kRowCands) / sizeof(int)); ++cand) {
      const int rows = cand < 0 ? 0 : kRowCands[cand];
      int r = 0;
      (void)stencil_grid(plan->Np, plan->Mp, &r, rows);
      if (rows > 0 && r != rows) continue;   // grid beyond the partials table
      StencilArgs<T> a = stencil_base<T>(plan, W.v[V_OV], W.v[V_OH], W.st);
      a.p_in = W.v[V_P0];
      a.q = W.v[V_Q];
      a.check_done = 0;
      a.rows = rows;
      const double us = time_launches([&] { launch_stencil<T>(ST_APPLY, a, s); }, 10, s);
      if (us < 0) return IRLSU_ERR_HIP;
      if (cand < 0 || us < best) {
        best = us;
        best_rows = rows;
      }
    }
    plan->tune_rows = best_rows;
    su = best;
    // 2) blocks of the CG update, with a state under which it runs through
    //    (rho = 1 and a single p.q partial of 1)
    const int nvec = stencil_blocks(plan);
    static const double one = 1.0;
    HIP_OK(hipMemcpyAsync(W.st.sc + SC_RHO, &one, sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(part_row_host(W.st, PR_PQ), &one, sizeof(double), hipMemcpyHostToDevice,
                          s));
    int best_upd = 0;
    best = 0.0;
    for (int cand = -1; cand < (int)(sizeof(kUpdateCands) / sizeof(int)); ++cand) {
      const int nb = cand < 0 ? axpy_blocks(nvec) : kUpdateCands[cand];
      if (nb > nvec) break;
      AxpyArgs<T> xa;
      xa.u = W.U;
      xa.d = W.v[V_D];
      xa.r = W.v[V_R];
      xa.p = W.v[V_P0];
      xa.q = W.v[V_Q];
      xa.n = (int64_t)npx;
      xa.nparts_pq = 1;
      xa.nparts_out = nvec;
      xa.iter = 0;
      xa.st = W.st;
      const double us = time_launches([&] { launch_axpy<T>(xa, s, nb); }, 10, s);
      if (us < 0) return IRLSU_ERR_HIP;
      if (cand < 0 || us < best) {
        best = us;
        best_upd = cand < 0 ? 0 : nb;
      }
    }
    plan->tune_update = best_upd;
    uu = best;
    // 3) product tiles of the 16-bit MFMA forms
    plan->tune_small = 0;
    if (!plan->fast && plan->opsz == 2) {
      best = 0.0;
      int best_small = 0;
      for (int small = 0; small < 2; ++small) {
        plan->tune_small = small;
        const PrecondArgs pa = precond_args<T>(plan, W, W.v[V_R], W.v[V_Z], nullptr, 0, 0);
        const double us = time_launches([&] { launch_precond(pa, s); }, 5, s);
        if (us < 0) return IRLSU_ERR_HIP;
        if (small == 0 || us < best) {
          best = us;
          best_small = small;
        }
      }
      plan->tune_small = best_small;
      pu = best;
    }
    HIP_OK(hipMemsetAsync(W.st.sc, 0, SC_COUNT * sizeof(double), s));
    HIP_OK(hipMemsetAsync(W.st.fl, 0, FL_COUNT * sizeof(int32_t), s));
    HIP_OK(hipStreamSynchronize(s));
    return IRLSU_OK;
  };
  st = plan->elem == 8 ? go(double{}) : go(float{});
  if (st != IRLSU_OK) return st;
  TuneEntry e = key;
  e.stencil_rows = plan->tune_rows;
  e.update_blocks = plan->tune_update;
  e.small_tiles = plan->tune_small;
  e.stencil_us = su;
  e.update_us = uu;
  e.precond_us = pu;
  if (cache_path) {
    tune_cache_put(cache, e);
    if (!tune_cache_write(cache_path, cache)) return IRLSU_ERR_INVALID_ARG;
  }
  put_tune(out, e.stencil_rows, e.update_blocks, e.small_tiles, 0, su, uu, pu);
  return IRLSU_OK;
}

irlsu_status irlsu_batch_autotune(irlsu_batch* b, const char* cache_path, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  if (!b) return IRLSU_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < b->ws_bytes) return IRLSU_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  const std::string arch = device_arch(dev);
  std::vector<TuneEntry> cache = tune_cache_read(cache_path);
  const int nt = b->ntiles;
  std::vector<int> rows(nt, 0);
  std::map<std::pair<int64_t, int64_t>, int> chosen;
  for (int t = 0; t < nt; ++t) {
    const auto shape = std::make_pair(b->N[t], b->M[t]);
    auto it = chosen.find(shape);
    if (it != chosen.end()) {
      rows[t] = it->second;
      continue;
    }
    TuneEntry key;
    key.kind = "batch_tile";
    key.arch = arch;
    key.N = b->N[t];
    key.M = b->M[t];
    key.precision = b->prec;
    key.form = b->fast[t] ? IRLSU_PLAN_FAST : 0;
    if (const TuneEntry* e = tune_cache_find(cache, key)) {
      rows[t] = e->stencil_rows;
      chosen[shape] = rows[t];
      continue;
    }
    // the tile's stencil alone on its own (zeroed) vectors; partials from 0
    const TileWs w = carve_tile(b, workspace, t);
    const size_t npx = (size_t)b->Np[t] * (size_t)b->Mp[t];
    for (int v : {2, 4, 10, 11}) HIP_OK(hipMemsetAsync(w.v[v], 0, npx * sizeof(float), s));
    DevState st = tile_state(b, workspace, t);
    st.off = 0;
    StencilArgs<float> a;
    std::memset(&a, 0, sizeof(a));
    a.Ov = w.v[10];
    a.Oh = w.v[11];
    a.p_in = w.v[2];
    a.q = w.v[4];
    a.N = b->N[t];
    a.M = b->M[t];
    a.Np = b->Np[t];
    a.ld = b->Mp[t];
    a.st = st;
    int best_rows = 0;
    double best = 0.0;
    for (int cand = -1; cand < (int)(sizeof(kRowCands) / sizeof(int)); ++cand) {
      const int r0 = cand < 0 ? 0 : kRowCands[cand];
      int r = 0;
      (void)stencil_grid(a.Np, a.ld, &r, r0);
      if (r0 > 0 && r != r0) continue;
      a.rows = r0;
      const double us = time_launches([&] { launch_stencil<float>(ST_APPLY, a, s); }, 10, s);
      if (us < 0) return IRLSU_ERR_HIP;
      if (cand < 0 || us < best) {
        best = us;
        best_rows = r0;
      }
    }
    rows[t] = best_rows;
    chosen[shape] = best_rows;
    TuneEntry e = key;
    e.stencil_rows = best_rows;
    e.stencil_us = best;
    tune_cache_put(cache, e);
  }
  std::vector<int32_t> st_start;
  if (batch_grids(b, rows, st_start) > kMaxPartials) {
    // the tuned grids need more partials than the table holds: defaults
    (void)batch_grids(b, std::vector<int>(nt, 0), st_start);
  }
  HIP_OK(hipMemcpy(b->d_st_start, st_start.data(), st_start.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
  if (cache_path && !tune_cache_write(cache_path, cache)) return IRLSU_ERR_INVALID_ARG;
  return IRLSU_OK;
}
