// Adjoint of the converged IRLS system (frozen weights): for a loss with
// dL/dU = gU, lambda solves D^T Omega D lambda = gU - mean(gU) (one extra PCG
// solve with the forward kernels), then per edge
//   g_Omega = -(D lambda) r,   g_C = omega g_Omega,   g_G = Omega (D lambda),
// with r = DU - G, omega = 1 / max(|r|, eps), Omega = C omega, and
// g_X = D^T g_G (the residue map W has derivative 1 away from its jumps).
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
    st.fl[FL_ITERS] = 0;
    st.fl[FL_STATUS] = 0;
  }
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
  auto edge = [&](int64_t o0, int64_t o1, double g, double c, double& gc, double& gg) {
    const double r = a.U[o1] - a.U[o0] - g;
    const double ar = fabs(r);
    const double om = 1.0 / (ar > eps ? ar : eps);
    const double dl = a.lam[o1] - a.lam[o0];
    gc = om * (-dl * r);
    gg = c * om * dl;
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

template void launch_adjoint_rhs<float>(const float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        float*, DevState, double, hipStream_t);
template void launch_adjoint_rhs<double>(const double*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                         double*, DevState, double, hipStream_t);
template void launch_adjoint_edges<float>(const AdjEdgeArgs<float>&, hipStream_t);
template void launch_adjoint_edges<double>(const AdjEdgeArgs<double>&, hipStream_t);

}  // namespace irlsu
