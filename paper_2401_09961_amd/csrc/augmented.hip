// The paper's augmented form in (U, V^v, V^h) (Algorithm 1 with the linear
// system of Proposition 1 solved by Algorithm 2): for weights
// W = sqrt(C^2 V^2 + delta^2) (the closed-form weight step), the symmetric
// system
//   [ D^T D / tau      -D^T / tau            ] [U]   [ D^T G / tau ]
//   [ -D / tau    diag(C^2 / W) + I / tau    ] [V] = [ -G / tau    ]
// preconditioned by blkdiag(tau L^+, (C^2 / W + 1 / tau)^-1) (the block
// preconditioner of Section 3.3; L^+ by the plan's cosine-basis solve).
// Every vector of the solve is a triple (u, v, h) of Np x ld arrays, the
// slack blocks stored on the padded edge layout (zero where no edge).
#include "kernels.hpp"

namespace irlsu {

namespace {

template <class T>
struct EdgeIdx {
  int64_t N, M, ld;
  __device__ bool vert(int64_t i, int64_t j) const { return i >= 0 && i + 1 < N && j >= 0 && j < M; }
  __device__ bool horz(int64_t i, int64_t j) const { return i >= 0 && i < N && j >= 0 && j + 1 < M; }
};

// ev = u(i+1,j) - u(i,j) - v(i,j) on a vertical edge, eh likewise; 0 off the grid
template <class T>
__device__ __forceinline__ double ev_at(const AugVec<T>& x, const EdgeIdx<T>& g, int64_t i,
                                        int64_t j) {
  if (!g.vert(i, j)) return 0.0;
  const int64_t o = i * g.ld + j;
  return (double)x.u[o + g.ld] - (double)x.u[o] - (double)x.v[o];
}
template <class T>
__device__ __forceinline__ double eh_at(const AugVec<T>& x, const EdgeIdx<T>& g, int64_t i,
                                        int64_t j) {
  if (!g.horz(i, j)) return 0.0;
  const int64_t o = i * g.ld + j;
  return (double)x.u[o + 1] - (double)x.u[o] - (double)x.h[o];
}

// (A x) at pixel (i, j): U block and the slack blocks of the edges below /
// right of the pixel.
template <class T>
__device__ __forceinline__ void apply_at(const AugArgs<T>& a, const AugVec<T>& x, int64_t i,
                                         int64_t j, double& qu, double& qv, double& qh) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  const double it = 1.0 / a.tau;
  const int64_t o = i * a.ld + j;
  qu = (-ev_at(x, g, i, j) + ev_at(x, g, i - 1, j) - eh_at(x, g, i, j) + eh_at(x, g, i, j - 1)) * it;
  qv = 0.0;
  qh = 0.0;
  if (g.vert(i, j))
    qv = -((double)x.u[o + a.ld] - (double)x.u[o]) * it + ((double)a.dv[o] + it) * (double)x.v[o];
  if (g.horz(i, j))
    qh = -((double)x.u[o + 1] - (double)x.u[o]) * it + ((double)a.dh[o] + it) * (double)x.h[o];
}

}  // namespace

// Weights W = sqrt(C^2 V^2 + delta^2) as d = C^2 / W on every edge, with
// partial F_delta(U, V) (sum sqrt(C^2 V^2 + delta^2) + |DU - G - V|^2 / 2 tau)
// and L1(U) = sum C |DU - G|.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_weights_kernel(AugArgs<T> a, AugVec<T> x) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  double acc[2] = {0.0, 0.0};
  const int64_t n = a.Np * a.ld;
  const double dl2 = a.delta * a.delta;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    double dv = 0.0, dh = 0.0;
    if (g.vert(i, j)) {
      const double c = (double)a.Cv[k], v = (double)x.v[k], gg = (double)a.Gv[k];
      const double w = sqrt(c * c * v * v + dl2);
      dv = c * c / w;
      const double r = (double)x.u[k + a.ld] - (double)x.u[k] - gg;
      acc[0] += w + (r - v) * (r - v) / (2.0 * a.tau);
      acc[1] += c * fabs(r);
    }
    if (g.horz(i, j)) {
      const double c = (double)a.Ch[k], v = (double)x.h[k], gg = (double)a.Gh[k];
      const double w = sqrt(c * c * v * v + dl2);
      dh = c * c / w;
      const double r = (double)x.u[k + 1] - (double)x.u[k] - gg;
      acc[0] += w + (r - v) * (r - v) / (2.0 * a.tau);
      acc[1] += c * fabs(r);
    }
    a.dv[k] = (T)dv;
    a.dh[k] = (T)dh;
  }
  const int slots[2] = {PT_A, PT_B};
  write_partials<2>(a.st, slots, acc, (int)blockIdx.x);
}

// Right-hand side (D^T G / tau, -G^v / tau, -G^h / tau), partial ||b||^2;
// and the starting point V^0 = D U^0 - G with U^0 = 0 when init is set.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_rhs_kernel(AugArgs<T> a, AugVec<T> b, AugVec<T> x,
                                                          int init) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  double acc[1] = {0.0};
  const int64_t n = a.Np * a.ld;
  const double it = 1.0 / a.tau;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    double bu = 0.0;
    if (i < a.N && j < a.M) {
      if (g.vert(i, j)) bu -= (double)a.Gv[k];
      if (g.vert(i - 1, j)) bu += (double)a.Gv[k - a.ld];
      if (g.horz(i, j)) bu -= (double)a.Gh[k];
      if (g.horz(i, j - 1)) bu += (double)a.Gh[k - 1];
    }
    const double bv = g.vert(i, j) ? -(double)a.Gv[k] * it : 0.0;
    const double bh = g.horz(i, j) ? -(double)a.Gh[k] * it : 0.0;
    const T tu = (T)(bu * it), tv = (T)bv, th = (T)bh;
    b.u[k] = tu;
    b.v[k] = tv;
    b.h[k] = th;
    acc[0] += (double)tu * (double)tu + (double)tv * (double)tv + (double)th * (double)th;
    if (init) {
      x.u[k] = (T)0;
      x.v[k] = g.vert(i, j) ? (T)(-(double)a.Gv[k]) : (T)0;
      x.h[k] = g.horz(i, j) ? (T)(-(double)a.Gh[k]) : (T)0;
    }
  }
  const int slots[1] = {PR_BB};
  write_partials<1>(a.st, slots, acc, (int)blockIdx.x);
}

// r = b - A x, partial ||r||^2 (all three blocks) and sum r_u.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_resid_kernel(AugArgs<T> a, AugVec<T> x, AugVec<T> b,
                                                            AugVec<T> r, int check_done) {
  if (check_done && a.st.fl[FL_DONE]) return;
  double acc[2] = {0.0, 0.0};
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    double qu = 0.0, qv = 0.0, qh = 0.0;
    if (i < a.N && j < a.M) apply_at(a, x, i, j, qu, qv, qh);
    const T ru = (T)((double)b.u[k] - qu), rv = (T)((double)b.v[k] - qv),
            rh = (T)((double)b.h[k] - qh);
    r.u[k] = ru;
    r.v[k] = rv;
    r.h[k] = rh;
    acc[0] += (double)ru * (double)ru + (double)rv * (double)rv + (double)rh * (double)rh;
    acc[1] += (double)ru;
  }
  const int slots[2] = {PR_RR, PR_RSUM};
  write_partials<2>(a.st, slots, acc, (int)blockIdx.x);
}

// Slack blocks of the preconditioner, z = r / (C^2 / W + 1 / tau), partial
// z . r of those blocks.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_vprecond_kernel(AugArgs<T> a, AugVec<T> r,
                                                               AugVec<T> z) {
  if (a.st.fl[FL_DONE]) return;
  double acc[1] = {0.0};
  const int64_t n = a.Np * a.ld;
  const double it = 1.0 / a.tau;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const T zv = (T)((double)r.v[k] / ((double)a.dv[k] + it));
    const T zh = (T)((double)r.h[k] / ((double)a.dh[k] + it));
    z.v[k] = zv;
    z.h[k] = zh;
    acc[0] += (double)zv * (double)r.v[k] + (double)zh * (double)r.h[k];
  }
  const int slots[1] = {PR_AUX};
  write_partials<1>(a.st, slots, acc, (int)blockIdx.x);
}

// rho = tau (z_u . r_u) + z_v . r_v; beta = rho / rho_old (0 at l = 0);
// p = (tau z_u, z_v) + beta p.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_pupdate_kernel(AugArgs<T> a, AugVec<T> z,
                                                              AugVec<T> p, int iter, int nparts_u,
                                                              int nparts_v) {
  if (a.st.fl[FL_DONE]) return;
  const double rho = a.tau * reduce_slot(a.st, PR_ZR, nparts_u) + reduce_slot(a.st, PR_AUX, nparts_v);
  double beta = 0.0;
  if (iter > 0) beta = rho / a.st.sc[SC_RHO + ((iter - 1) & 1)];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st.sc[SC_RHO + (iter & 1)] = rho;
    a.st.sc[SC_BETA] = beta;
  }
  const T tt = (T)a.tau, bt = (T)beta;
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    p.u[k] = tt * z.u[k] + bt * p.u[k];
    p.v[k] = z.v[k] + bt * p.v[k];
    p.h[k] = z.h[k] + bt * p.h[k];
  }
}

// q = A p, partial p . q.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_apply_kernel(AugArgs<T> a, AugVec<T> p, AugVec<T> q) {
  if (a.st.fl[FL_DONE]) return;
  double acc[1] = {0.0};
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    double qu = 0.0, qv = 0.0, qh = 0.0;
    if (i < a.N && j < a.M) apply_at(a, p, i, j, qu, qv, qh);
    const T tu = (T)qu, tv = (T)qv, th = (T)qh;
    q.u[k] = tu;
    q.v[k] = tv;
    q.h[k] = th;
    acc[0] += (double)p.u[k] * (double)tu + (double)p.v[k] * (double)tv + (double)p.h[k] * (double)th;
  }
  const int slots[1] = {PR_PQ};
  write_partials<1>(a.st, slots, acc, (int)blockIdx.x);
}

// alpha = rho / p.q; x += alpha p; r -= alpha q; partial ||r||^2, sum r_u.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_axpy_kernel(AugArgs<T> a, AugVec<T> x, AugVec<T> r,
                                                           AugVec<T> p, AugVec<T> q, int iter,
                                                           int nparts_pq) {
  if (a.st.fl[FL_DONE]) return;
  const double pq = reduce_slot(a.st, PR_PQ, nparts_pq);
  const double rho = a.st.sc[SC_RHO + (iter & 1)];
  if (!(pq > 0.0) || !(rho >= 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.st.fl[FL_STATUS] |= 1;
      a.st.fl[FL_DONE] = 1;
    }
    return;
  }
  const double alpha = rho / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st.sc[SC_ALPHA + (iter & 1)] = alpha;
    a.st.fl[FL_ITERS] = iter + 1;
  }
  const T al = (T)alpha;
  double acc[2] = {0.0, 0.0};
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    x.u[k] += al * p.u[k];
    x.v[k] += al * p.v[k];
    x.h[k] += al * p.h[k];
    const T ru = r.u[k] - al * q.u[k], rv = r.v[k] - al * q.v[k], rh = r.h[k] - al * q.h[k];
    r.u[k] = ru;
    r.v[k] = rv;
    r.h[k] = rh;
    acc[0] += (double)ru * (double)ru + (double)rv * (double)rv + (double)rh * (double)rh;
    acc[1] += (double)ru;
  }
  const int slots[2] = {PR_RR, PR_RSUM};
  write_partials<2>(a.st, slots, acc, (int)blockIdx.x);
}

// U -= mean(U) over the valid pixels (Algorithm 1's last step).
template <class T>
__global__ __launch_bounds__(kThreads) void aug_sum_kernel(AugArgs<T> a, const T* u) {
  double acc[1] = {0.0};
  const int64_t n = a.N * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads)
    if (k % a.ld < a.M) acc[0] += (double)u[k];
  const int slots[1] = {PT_C};
  write_partials<1>(a.st, slots, acc, (int)blockIdx.x);
}

template <class T>
__global__ __launch_bounds__(kThreads) void aug_center_kernel(AugArgs<T> a, T* u, int nparts) {
  const double mean = reduce_slot(a.st, PT_C, nparts) / ((double)a.N * (double)a.M);
  const int64_t n = a.N * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads)
    if (k % a.ld < a.M) u[k] = (T)((double)u[k] - mean);
}

// ---- sufficient-decrease guard of Theorem 3 ---------------------------------
// DU - G - V on the vertical / horizontal edge at (i, j); 0 off the grid.
template <class T>
__device__ __forceinline__ double gev_at(const AugArgs<T>& a, const AugVec<T>& x,
                                         const EdgeIdx<T>& g, int64_t i, int64_t j) {
  return g.vert(i, j) ? ev_at(x, g, i, j) - (double)a.Gv[i * g.ld + j] : 0.0;
}
template <class T>
__device__ __forceinline__ double geh_at(const AugArgs<T>& a, const AugVec<T>& x,
                                         const EdgeIdx<T>& g, int64_t i, int64_t j) {
  return g.horz(i, j) ? eh_at(x, g, i, j) - (double)a.Gh[i * g.ld + j] : 0.0;
}

// Candidate x~ = x - grad / L of (eq:candidate-gd-step), the gradient of the
// (prob:alt1) objective at the current weights (d = C^2 / W):
//   grad_U = D^T (DU - G - V) / tau,  grad_V = d V - (DU - G - V) / tau.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_cand_kernel(AugArgs<T> a, AugVec<T> x,
                                                           AugVec<T> c) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  const int64_t n = a.Np * a.ld;
  const double it = 1.0 / a.tau, invL = a.st.sc[SC_INVL];
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    double cu = 0.0, cv = 0.0, ch = 0.0;
    if (i < a.N && j < a.M) {
      const double ev = gev_at(a, x, g, i, j), eh = geh_at(a, x, g, i, j);
      const double gu =
          (-ev + gev_at(a, x, g, i - 1, j) - eh + geh_at(a, x, g, i, j - 1)) * it;
      cu = (double)x.u[k] - gu * invL;
      if (g.vert(i, j)) {
        const double v = (double)x.v[k];
        cv = v - ((double)a.dv[k] * v - ev * it) * invL;
      }
      if (g.horz(i, j)) {
        const double h = (double)x.h[k];
        ch = h - ((double)a.dh[k] * h - eh * it) * invL;
      }
    }
    c.u[k] = (T)cu;
    c.v[k] = (T)cv;
    c.h[k] = (T)ch;
  }
}

// Block maximum of v over the block's threads (thread 0 returns it).
__device__ __forceinline__ double block_max(double v) {
  __shared__ double sm[kThreads];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  return sm[0];
}

// C_max of Theorem 3 over the edge weights: one maximum per block as partial.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_cmax_kernel(AugArgs<T> a) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  double m = 0.0;
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    if (g.vert(i, j)) m = fmax(m, (double)a.Cv[k]);
    if (g.horz(i, j)) m = fmax(m, (double)a.Ch[k]);
  }
  m = block_max(m);
  if (threadIdx.x == 0) part_row(a.st, PR_AUX)[blockIdx.x] = m;
}

// 1 / L, L = 12 / tau + C_max^2 / delta (Theorem 3), into SC_INVL.
__global__ __launch_bounds__(kThreads) void aug_invl_kernel(DevState st, int nparts, double tau,
                                                           double delta) {
  const double* p = part_row(st, PR_AUX);
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) m = fmax(m, p[i]);
  m = block_max(m);
  if (threadIdx.x == 0) st.sc[SC_INVL] = 1.0 / (12.0 / tau + m * m / delta);
}

// Partial of the (prob:alt1) objective of x at the current weights,
// 1/2 sum ((C^2 V^2 + delta^2) / W + W) + sum (DU - G - V)^2 / (2 tau), with
// W = C^2 / d from the stored d (both guard evaluations use the same W).
template <class T>
__global__ __launch_bounds__(kThreads) void aug_hval_kernel(AugArgs<T> a, AugVec<T> x) {
  const EdgeIdx<T> g{a.N, a.M, a.ld};
  double acc[1] = {0.0};
  const int64_t n = a.Np * a.ld;
  const double dl2 = a.delta * a.delta, h2t = 0.5 / a.tau;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / a.ld, j = k % a.ld;
    if (g.vert(i, j)) {
      const double c = (double)a.Cv[k], d = (double)a.dv[k], v = (double)x.v[k];
      const double w = c * c / d, e = gev_at(a, x, g, i, j);
      acc[0] += 0.5 * (d * v * v + dl2 / w + w) + h2t * e * e;
    }
    if (g.horz(i, j)) {
      const double c = (double)a.Ch[k], d = (double)a.dh[k], v = (double)x.h[k];
      const double w = c * c / d, e = geh_at(a, x, g, i, j);
      acc[0] += 0.5 * (d * v * v + dl2 / w + w) + h2t * e * e;
    }
  }
  const int slots[1] = {PR_AUX};
  write_partials<1>(a.st, slots, acc, (int)blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void aug_store_kernel(DevState st, int nparts, int sc) {
  const double v = reduce_slot(st, PR_AUX, nparts);
  if (threadIdx.x == 0) st.sc[sc] = v;
}

// mode 1: keep the solve's x when its objective is no larger than the
// candidate's (the condition of Theorem 3), else x = c; mode 2: x = c.
template <class T>
__global__ __launch_bounds__(kThreads) void aug_guard_kernel(AugArgs<T> a, AugVec<T> x,
                                                            AugVec<T> c, int mode) {
  const bool take = mode == 2 || !(a.st.sc[SC_SNEW] <= a.st.sc[SC_SOLD]);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.st.fl[FL_GUARD] = take ? 2 : 1;
  if (!take) return;
  const int64_t n = a.Np * a.ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    x.u[k] = c.u[k];
    x.v[k] = c.v[k];
    x.h[k] = c.h[k];
  }
}

// Objectives into scalars: F_delta -> SC_H, L1 -> SC_L1.
__global__ __launch_bounds__(kThreads) void aug_objectives_kernel(DevState st, int nparts) {
  const double f = reduce_slot(st, PT_A, nparts);
  const double l1 = reduce_slot(st, PT_B, nparts);
  if (threadIdx.x == 0) {
    st.sc[SC_H] = f;
    st.sc[SC_L1] = l1;
  }
}

// ||b||^2 into SC_BB (nparts > 0; the right-hand side is fixed, later
// solves keep the value: its partial slot is reused), tolerance, fresh PCG
// flags.
__global__ __launch_bounds__(kThreads) void aug_start_kernel(DevState st, int nparts, double tol2) {
  const double bb = nparts > 0 ? reduce_slot(st, PR_BB, nparts) : 0.0;
  if (threadIdx.x == 0) {
    if (nparts > 0) st.sc[SC_BB] = bb;
    st.sc[SC_TOL2] = tol2;
    st.fl[FL_DONE] = 0;
    st.fl[FL_DPEND] = 0;
    st.fl[FL_ITERS] = 0;
  }
}

template <class T>
int aug_launch(int op, const AugArgs<T>& a, const AugVec<T>& x, const AugVec<T>& y,
               const AugVec<T>& z, const AugVec<T>& w, int i0, int i1, int i2, double d0,
               hipStream_t s) {
  const int nb = elementwise_blocks(a.Np * a.ld);
  const dim3 g(nb), b(kThreads);
  switch (op) {
    case AUG_WEIGHTS:
      hipLaunchKernelGGL(aug_weights_kernel<T>, g, b, 0, s, a, x);
      hipLaunchKernelGGL(aug_objectives_kernel, dim3(1), b, 0, s, a.st, nb);
      break;
    case AUG_RHS:  // x = start, y = b
      hipLaunchKernelGGL(aug_rhs_kernel<T>, g, b, 0, s, a, y, x, i0);
      hipLaunchKernelGGL(aug_start_kernel, dim3(1), b, 0, s, a.st, nb, d0);
      break;
    case AUG_START:
      hipLaunchKernelGGL(aug_start_kernel, dim3(1), b, 0, s, a.st, i0, d0);
      break;
    case AUG_RESID:  // x, b -> r (y = b, z = r)
      hipLaunchKernelGGL(aug_resid_kernel<T>, g, b, 0, s, a, x, y, z, i0);
      break;
    case AUG_VPRECOND:  // r -> z (slack blocks)
      hipLaunchKernelGGL(aug_vprecond_kernel<T>, g, b, 0, s, a, x, y);
      break;
    case AUG_PUPDATE:  // z, p
      hipLaunchKernelGGL(aug_pupdate_kernel<T>, g, b, 0, s, a, x, y, i0, i1, i2);
      break;
    case AUG_APPLY:  // p -> q
      hipLaunchKernelGGL(aug_apply_kernel<T>, g, b, 0, s, a, x, y);
      break;
    case AUG_AXPY:  // x, r, p, q
      hipLaunchKernelGGL(aug_axpy_kernel<T>, g, b, 0, s, a, x, y, z, w, i0, i1);
      break;
    case AUG_CENTER:
      hipLaunchKernelGGL(aug_sum_kernel<T>, g, b, 0, s, a, x.u);
      hipLaunchKernelGGL(aug_center_kernel<T>, g, b, 0, s, a, x.u, nb);
      break;
    case AUG_CAND:  // x -> y
      hipLaunchKernelGGL(aug_cand_kernel<T>, g, b, 0, s, a, x, y);
      break;
    case AUG_INVL:
      hipLaunchKernelGGL(aug_cmax_kernel<T>, g, b, 0, s, a);
      hipLaunchKernelGGL(aug_invl_kernel, dim3(1), b, 0, s, a.st, nb, a.tau, a.delta);
      break;
    case AUG_HVAL:  // x -> sc[i0]
      hipLaunchKernelGGL(aug_hval_kernel<T>, g, b, 0, s, a, x);
      hipLaunchKernelGGL(aug_store_kernel, dim3(1), b, 0, s, a.st, nb, i0);
      break;
    case AUG_GUARD:  // x, y = candidate; i0 = mode
      hipLaunchKernelGGL(aug_guard_kernel<T>, g, b, 0, s, a, x, y, i0);
      break;
  }
  return nb;
}

template int aug_launch<float>(int, const AugArgs<float>&, const AugVec<float>&,
                               const AugVec<float>&, const AugVec<float>&, const AugVec<float>&,
                               int, int, int, double, hipStream_t);
template int aug_launch<double>(int, const AugArgs<double>&, const AugVec<double>&,
                                const AugVec<double>&, const AugVec<double>&,
                                const AugVec<double>&, int, int, int, double, hipStream_t);

}  // namespace irlsu
