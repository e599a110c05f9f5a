// Adjoint of the converged IRLS system.  Frozen weights: for a loss with
// dL/dU = gU, lambda solves D^T Omega D lambda = gU - mean(gU) (one extra PCG
// solve with the forward kernels), then per edge
//   g_Omega = -(D lambda) r,   g_C = omega g_Omega,   g_G = Omega (D lambda),
// with r = DU - G, omega = 1 / max(|r|, eps), Omega = C omega, and
// g_X = D^T g_G (the residue map W has derivative 1 away from its jumps).
// Full implicit derivative of the Huber minimiser: the stationarity condition
// D^T (C h_eps'(r)) = 0 differentiates with the Hessian weights kappa = C /
// eps on the quadratic zone |r| < eps (0 off it): lambda solves
// D^T kappa D lambda = gU (projected, see below), then
//   g_G = kappa (D lambda),   g_C = -h_eps'(r) (D lambda),   g_X = D^T g_G.
// Pixels with no quadratic-zone edge (where the minimiser is not unique) are
// left out: gU is taken as zero there and lambda = 0 there, lambda has mean
// zero over the other pixels.
#include "kernels.hpp"

namespace irlsu {

// Sum of gU over the valid pixels (for the mean).
template <class T>
__global__ __launch_bounds__(kThreads) void adj_rhs_sum_kernel(const T* g, int64_t ldg, int64_t N,
                                                              int64_t M, DevState st) {
  double acc[1] = {0.0};
  const int64_t n = N * M;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / M, j = k % M;
    acc[0] += (double)g[i * ldg + j];
  }
  const int slots[1] = {PR_AUX};
  write_partials<1>(st, slots, acc, linear_block());
}

// b = gU - mean(gU) in the internal layout (zero padding), partial ||b||^2.
template <class T>
__global__ __launch_bounds__(kThreads) void adj_rhs_write_kernel(const T* g, int64_t ldg, int64_t N,
                                                                int64_t M, int64_t Np, int64_t ld,
                                                                T* b, DevState st, int nparts) {
  const double mean = reduce_slot(st, PR_AUX, nparts) / ((double)N * (double)M);
  double acc[1] = {0.0};
  const int64_t n = Np * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / ld, j = k % ld;
    T v = (T)0;
    if (i < N && j < M) v = (T)((double)g[i * ldg + j] - mean);
    b[k] = v;
    acc[0] += (double)v * (double)v;
  }
  const int slots[1] = {PR_BB};
  write_partials<1>(st, slots, acc, linear_block());
}

__global__ __launch_bounds__(kThreads) void adj_finalize_kernel(DevState st, int nparts, double tol2) {
  const double bb = reduce_slot(st, PR_BB, nparts);
  if (threadIdx.x == 0) {
    st.sc[SC_BB] = bb;
    st.sc[SC_TOL2] = tol2;
    st.fl[FL_DONE] = 0;
    st.fl[FL_DPEND] = 0;
    st.fl[FL_ITERS] = 0;
    st.fl[FL_STATUS] = 0;
  }
}

// ---- full implicit derivative: Hessian weights, projected right-hand side
template <class T>
__global__ __launch_bounds__(kThreads) void adj_hessian_kernel(const double* U, const T* Gv,
                                                              const T* Gh, const T* Cv,
                                                              const T* Ch, double eps, int64_t N,
                                                              int64_t M, int64_t Np, int64_t ld,
                                                              T* Kv, T* Kh) {
  const int64_t n = Np * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / ld, j = k % ld;
    double kv = 0.0, kh = 0.0;
    if (i + 1 < N && j < M) {
      const double r = U[k + ld] - U[k] - (double)Gv[k];
      if (fabs(r) < eps) kv = (double)Cv[k] / eps;
    }
    if (i < N && j + 1 < M) {
      const double r = U[k + 1] - U[k] - (double)Gh[k];
      if (fabs(r) < eps) kh = (double)Ch[k] / eps;
    }
    Kv[k] = (T)kv;
    Kh[k] = (T)kh;
  }
}

// true when pixel (i, j) has no edge of positive Hessian weight
template <class T>
__device__ __forceinline__ bool left_out(const T* Kv, const T* Kh, int64_t i, int64_t j, int64_t N,
                                         int64_t M, int64_t ld) {
  const int64_t o = i * ld + j;
  if (i + 1 < N && Kv[o] > (T)0) return false;
  if (i > 0 && Kv[o - ld] > (T)0) return false;
  if (j + 1 < M && Kh[o] > (T)0) return false;
  if (j > 0 && Kh[o - 1] > (T)0) return false;
  return true;
}

// sum and count of gU (double) over the kept pixels
template <class T, class G>
__global__ __launch_bounds__(kThreads) void adj_kept_sum_kernel(const G* g, int64_t ldg, int64_t N,
                                                               int64_t M, int64_t ld, const T* Kv,
                                                               const T* Kh, DevState st) {
  double acc[2] = {0.0, 0.0};
  const int64_t n = N * M;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / M, j = k % M;
    if (!left_out(Kv, Kh, i, j, N, M, ld)) {
      acc[0] += (double)g[i * ldg + j];
      acc[1] += 1.0;
    }
  }
  const int slots[2] = {PR_AUX, PT_D};
  write_partials<2>(st, slots, acc, linear_block());
}

template <class T>
__global__ __launch_bounds__(kThreads) void adj_rhs_write_kept_kernel(
    const T* g, int64_t ldg, int64_t N, int64_t M, int64_t Np, int64_t ld, const T* Kv,
    const T* Kh, T* b, DevState st, int nparts) {
  const double cnt = reduce_slot(st, PT_D, nparts);
  const double mean = cnt > 0.0 ? reduce_slot(st, PR_AUX, nparts) / cnt : 0.0;
  double acc[1] = {0.0};
  const int64_t n = Np * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / ld, j = k % ld;
    T v = (T)0;
    if (i < N && j < M && !left_out(Kv, Kh, i, j, N, M, ld))
      v = (T)((double)g[i * ldg + j] - mean);
    b[k] = v;
    acc[0] += (double)v * (double)v;
  }
  const int slots[1] = {PR_BB};
  write_partials<1>(st, slots, acc, linear_block());
}

__global__ __launch_bounds__(kThreads) void adj_mean_kernel(DevState st, int nparts) {
  const double cnt = reduce_slot(st, PT_D, nparts);
  const double sum = reduce_slot(st, PR_AUX, nparts);
  if (threadIdx.x == 0) st.sc[SC_MEAN] = cnt > 0.0 ? sum / cnt : 0.0;
}

// Edge gradients and g_X = D^T g_G.  One thread per pixel; the edges above
// and to the left are recomputed from their endpoints.
template <class T>
__global__ __launch_bounds__(kThreads) void adj_edges_kernel(AdjEdgeArgs<T> a) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (i >= a.N || j >= a.M) return;
  const int64_t ld = a.ld;
  const int64_t o = i * ld + j;
  const double eps = a.eps;
  const bool implicit = a.Kv != nullptr;
  const double lm = implicit ? *a.lam_mean : 0.0;
  // lambda with the left-out pixels at 0 and mean zero over the others
  auto lam = [&](int64_t o1) -> double {
    if (!implicit) return a.lam[o1];
    return left_out(a.Kv, a.Kh, o1 / ld, o1 % ld, a.N, a.M, ld) ? 0.0 : a.lam[o1] - lm;
  };
  auto edge = [&](int64_t o0, int64_t o1, double g, double c, double& gc, double& gg) {
    const double r = a.U[o1] - a.U[o0] - g;
    const double ar = fabs(r);
    const double dl = lam(o1) - lam(o0);
    if (implicit) {
      const bool quad = ar < eps;
      gc = -(quad ? r / eps : (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0))) * dl;
      gg = quad ? c / eps * dl : 0.0;
    } else {
      const double om = 1.0 / (ar > eps ? ar : eps);
      gc = om * (-dl * r);
      gg = c * om * dl;
    }
  };
  double gx = 0.0;
  if (i + 1 < a.N) {
    double gc, gg;
    edge(o, o + ld, (double)a.Gv[o], (double)a.Cv[o], gc, gg);
    a.gCv[i * a.ldgcv + j] = (T)gc;
    gx -= gg;
  }
  if (j + 1 < a.M) {
    double gc, gg;
    edge(o, o + 1, (double)a.Gh[o], (double)a.Ch[o], gc, gg);
    a.gCh[i * a.ldgch + j] = (T)gc;
    gx -= gg;
  }
  if (i > 0) {
    double gc, gg;
    edge(o - ld, o, (double)a.Gv[o - ld], (double)a.Cv[o - ld], gc, gg);
    gx += gg;
  }
  if (j > 0) {
    double gc, gg;
    edge(o - 1, o, (double)a.Gh[o - 1], (double)a.Ch[o - 1], gc, gg);
    gx += gg;
  }
  if (a.gX) a.gX[i * a.ldgx + j] = (T)gx;
}

template <class T>
void launch_adjoint_rhs(const T* g, int64_t ldg, int64_t N, int64_t M, int64_t Np, int64_t ld,
                        T* b, DevState st, double tol2, hipStream_t s) {
  const int nb = elementwise_blocks(Np * ld);
  hipLaunchKernelGGL(adj_rhs_sum_kernel<T>, dim3(nb), dim3(kThreads), 0, s, g, ldg, N, M, st);
  hipLaunchKernelGGL(adj_rhs_write_kernel<T>, dim3(nb), dim3(kThreads), 0, s, g, ldg, N, M, Np, ld,
                     b, st, nb);
  hipLaunchKernelGGL(adj_finalize_kernel, dim3(1), dim3(kThreads), 0, s, st, nb, tol2);
}

template <class T>
void launch_adjoint_edges(const AdjEdgeArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.M + kThreads - 1) / kThreads), (unsigned)a.N);
  hipLaunchKernelGGL(adj_edges_kernel<T>, grid, dim3(kThreads), 0, s, a);
}

template <class T>
void launch_adjoint_hessian(const double* U, const T* Gv, const T* Gh, const T* Cv, const T* Ch,
                            double eps, int64_t N, int64_t M, int64_t Np, int64_t ld, T* Kv, T* Kh,
                            hipStream_t s) {
  hipLaunchKernelGGL(adj_hessian_kernel<T>, dim3(elementwise_blocks(Np * ld)), dim3(kThreads), 0,
                     s, U, Gv, Gh, Cv, Ch, eps, N, M, Np, ld, Kv, Kh);
}

template <class T>
void launch_adjoint_rhs_implicit(const T* g, int64_t ldg, int64_t N, int64_t M, int64_t Np,
                                 int64_t ld, const T* Kv, const T* Kh, T* b, DevState st,
                                 double tol2, hipStream_t s) {
  const int nb = elementwise_blocks(Np * ld);
  hipLaunchKernelGGL((adj_kept_sum_kernel<T, T>), dim3(nb), dim3(kThreads), 0, s, g, ldg, N, M,
                     ld, Kv, Kh, st);
  hipLaunchKernelGGL(adj_rhs_write_kept_kernel<T>, dim3(nb), dim3(kThreads), 0, s, g, ldg, N, M,
                     Np, ld, Kv, Kh, b, st, nb);
  hipLaunchKernelGGL(adj_finalize_kernel, dim3(1), dim3(kThreads), 0, s, st, nb, tol2);
}

template <class T>
void launch_adjoint_lam_mean(const double* lam, int64_t N, int64_t M, int64_t ld, const T* Kv,
                             const T* Kh, DevState st, hipStream_t s) {
  const int nb = elementwise_blocks(N * M);
  hipLaunchKernelGGL((adj_kept_sum_kernel<T, double>), dim3(nb), dim3(kThreads), 0, s, lam, ld, N,
                     M, ld, Kv, Kh, st);
  hipLaunchKernelGGL(adj_mean_kernel, dim3(1), dim3(kThreads), 0, s, st, nb);
}

#define IRLSU_ADJ_INST(T)                                                                      \
  template void launch_adjoint_hessian<T>(const double*, const T*, const T*, const T*, const T*, \
                                          double, int64_t, int64_t, int64_t, int64_t, T*, T*,   \
                                          hipStream_t);                                         \
  template void launch_adjoint_rhs_implicit<T>(const T*, int64_t, int64_t, int64_t, int64_t,    \
                                               int64_t, const T*, const T*, T*, DevState,       \
                                               double, hipStream_t);                            \
  template void launch_adjoint_lam_mean<T>(const double*, int64_t, int64_t, int64_t, const T*,  \
                                           const T*, DevState, hipStream_t);
IRLSU_ADJ_INST(float)
IRLSU_ADJ_INST(double)
#undef IRLSU_ADJ_INST

template void launch_adjoint_rhs<float>(const float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        float*, DevState, double, hipStream_t);
template void launch_adjoint_rhs<double>(const double*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                         double*, DevState, double, hipStream_t);
template void launch_adjoint_edges<float>(const AdjEdgeArgs<float>&, hipStream_t);
template void launch_adjoint_edges<double>(const AdjEdgeArgs<double>&, hipStream_t);

}  // namespace irlsu
