// Point-wise and reduction kernels of the IRLS + PCG path: setup of the
// wrapped gradients and edge weights, the IRLS weight step, the CG axpy,
// mean removal and the scalar finalisers.  All HBM-bound: one pass each,
// FP64 accumulation of every reduction through deterministic block sums.
#include "kernels.hpp"

namespace irlsu {

// ----------------------------------------------------------------------------
// Setup (Section 2): G = W(X_{i+1,j} - X_{ij}) etc. with W the residue in
// [-pi, pi), computed in FP64 with explicitly rounded operations so that the
// branch taken by floor() is the one the FP64 definition takes.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wrap_residue(double d) {
  const double kPi = 3.141592653589793;
  const double kTwoPi = 6.283185307179586;
  const double k = floor(__ddiv_rn(__dadd_rn(d, kPi), kTwoPi));
  return __dsub_rn(d, __dmul_rn(kTwoPi, k));
}

template <class T>
__global__ __launch_bounds__(kThreads) void setup_kernel(
    SetupArgs<T> a) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= a.ld) return;
  const int64_t N = a.N, M = a.M;
  const int64_t o = i * a.ld + j;
  T gv = 0, gh = 0, cv = 0, ch = 0;
  int bad = 0;
  if (i < N && j < M) {
    const double x0 = (double)a.X[i * a.ldx + j];
    if (!isfinite(x0)) bad |= 1;
    if (a.w) {
      const double w0 = (double)a.w[i * a.ldx + j];
      if (!isfinite(w0)) bad |= 1;
      else if (!(w0 > 0.0)) bad |= 2;
    }
    if (i + 1 < N) {
      const double x1 = (double)a.X[(i + 1) * a.ldx + j];
      gv = (T)wrap_residue(x1 - x0);
      if (a.Cv) {
        const T c = a.Cv[i * a.ldcv + j];
        if (!isfinite((double)c)) bad |= 1;
        else if (!((double)c > 0.0)) bad |= 2;
        cv = c;
      } else if (a.w) {
        const T w0 = a.w[i * a.ldx + j], w1 = a.w[(i + 1) * a.ldx + j];
        cv = w0 < w1 ? w0 : w1;
      } else {
        cv = (T)1;
      }
    }
    if (j + 1 < M) {
      const double x1 = (double)a.X[i * a.ldx + j + 1];
      gh = (T)wrap_residue(x1 - x0);
      if (a.Ch) {
        const T c = a.Ch[i * a.ldch + j];
        if (!isfinite((double)c)) bad |= 1;
        else if (!((double)c > 0.0)) bad |= 2;
        ch = c;
      } else if (a.w) {
        const T w0 = a.w[i * a.ldx + j], w1 = a.w[i * a.ldx + j + 1];
        ch = w0 < w1 ? w0 : w1;
      } else {
        ch = (T)1;
      }
    }
  }
  a.Gv[o] = gv;
  a.Gh[o] = gh;
  a.Cv_out[o] = cv;
  a.Ch_out[o] = ch;
  if (a.U) {
    double u = 0.0;
    if (a.U0 && i < N && j < M) {
      u = (double)a.U0[i * a.ldu0 + j];
      if (!isfinite(u)) bad |= 1;
    }
    a.U[o] = u;
  }
  if (bad) atomicOr(a.flags, bad);
}

// ----------------------------------------------------------------------------
// IRLS weight step: r = DU - G, Omega = C / max(|r|, eps), b = D^T (Omega G),
// partial sums of C|r|, C h_eps(r) and b^2.  One thread per pixel; the edges
// above and to the left are recomputed from cached neighbours.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double edge_omega(double c, double r, double eps) {
  const double a = fabs(r);
  return c / (a > eps ? a : eps);
}

template <class T>
__global__ __launch_bounds__(kThreads) void weights_kernel(WeightsArgs<T> a, int rows_per_block) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_block;
  int64_t i1 = i0 + rows_per_block;
  if (i1 > a.Np) i1 = a.Np;
  if (j < a.ld) {
    const int64_t ld = a.ld;
    const double eps = a.eps;
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t o = i * ld + j;
      const double u = a.U[o];
      const double ud = (i + 1 < a.Np) ? a.U[o + ld] : 0.0;
      const double ur = (j + 1 < ld) ? a.U[o + 1] : 0.0;
      const double gv = (double)a.Gv[o], gh = (double)a.Gh[o];
      const double cv = (double)a.Cv[o], ch = (double)a.Ch[o];
      const double rv = ud - u - gv;
      const double rh = ur - u - gh;
      const double ov = edge_omega(cv, rv, eps);
      const double oh = edge_omega(ch, rh, eps);
      double bsum = -ov * gv - oh * gh;
      if (i > 0) {
        const double gvu = (double)a.Gv[o - ld], cvu = (double)a.Cv[o - ld];
        bsum += edge_omega(cvu, u - a.U[o - ld] - gvu, eps) * gvu;
      }
      if (j > 0) {
        const double ghl = (double)a.Gh[o - 1], chl = (double)a.Ch[o - 1];
        bsum += edge_omega(chl, u - a.U[o - 1] - ghl, eps) * ghl;
      }
      if (a.want_model) {
        // S(U, Omega) = sum Omega r^2 / 2 + C^2 / (2 Omega) over the edges
        // present (C > 0): previous weights (as stored) and new weights
        auto model = [](double c, double om, double r) {
          return c > 0.0 ? 0.5 * om * r * r + 0.5 * c * c / om : 0.0;
        };
        acc[3] += model(cv, (double)a.Ov[o], rv) + model(ch, (double)a.Oh[o], rh);
        acc[4] += model(cv, ov, rv) + model(ch, oh, rh);
      }
      a.Ov[o] = (T)ov;
      a.Oh[o] = (T)oh;
      a.b[o] = (T)bsum;
      const double arv = fabs(rv), arh = fabs(rh);
      acc[0] += cv * arv + ch * arh;
      acc[1] += cv * (arv <= eps ? 0.5 * arv * arv / eps : arv - 0.5 * eps) +
                ch * (arh <= eps ? 0.5 * arh * arh / eps : arh - 0.5 * eps);
      const double bt = (double)(T)bsum;
      acc[2] += bt * bt;
    }
  }
  const int slots[5] = {PR_L1, PR_H, PR_BB, PT_D, PR_ZQ};
  write_partials<5>(a.st, slots, acc, linear_block());
}

// Finalise the weight step: objectives and ||b||^2 into scalars (and an
// optional user array), reset the PCG flags for the next solve.
__global__ __launch_bounds__(kThreads) void finalize_weights_kernel(
    DevState st, int nparts, double* out, double tol2, int want_model) {
  const double l1 = reduce_slot(st, PR_L1, nparts);
  const double h = reduce_slot(st, PR_H, nparts);
  const double bb = reduce_slot(st, PR_BB, nparts);
  const double s_old = want_model ? reduce_slot(st, PT_D, nparts) : 0.0;
  const double s_new = want_model ? reduce_slot(st, PR_ZQ, nparts) : 0.0;
  if (threadIdx.x == 0) {
    st.sc[SC_SOLD] = s_old;
    st.sc[SC_SNEW] = s_new;
    st.sc[SC_L1] = l1;
    st.sc[SC_H] = h;
    st.sc[SC_BB] = bb;
    st.sc[SC_TOL2] = tol2;
    st.fl[FL_DONE] = 0;
    st.fl[FL_DPEND] = 0;
    st.fl[FL_ITERS] = 0;
    if (out) {
      out[0] = l1;
      out[1] = h;
      out[2] = bb;
    }
  }
}

// ----------------------------------------------------------------------------
// CG update (Algorithm 2): alpha = rho / p.q, u += alpha p, r -= alpha q,
// partial ||r||^2 and sum r.  The prologue reduces the stencil's p.q partials
// (identically in every block) and stops on breakdown.
// ----------------------------------------------------------------------------
// Body shared by the single-image and the grouped (batched) launch: block lb
// of nb blocks working on one problem.
template <class T>
__device__ __forceinline__ void axpy_body(const AxpyArgs<T>& a, int lb, int nb) {
  if (a.st.fl[FL_DONE]) return;
  const double pq = reduce_slot(a.st, PR_PQ, a.nparts_pq);
  const double rho = a.st.sc[SC_RHO + (a.iter & 1)];
  if (!(pq > 0.0) || !(rho >= 0.0) || !isfinite(pq)) {
    if (lb == 0 && threadIdx.x == 0) {
      a.st.fl[FL_STATUS] |= 1;
      a.st.fl[FL_DONE] = 1;
    }
    return;
  }
  const double alpha = rho / pq;
  if (lb == 0 && threadIdx.x == 0) {
    a.st.sc[SC_ALPHA + (a.iter & 1)] = alpha;
    a.st.sc[SC_PQ] = pq;
    a.st.fl[FL_ITERS] += 1;  // counted on the device: iteration-independent launches
  }
  const T al = (T)alpha;
  double acc[2] = {0.0, 0.0};
  const int64_t n4 = a.n / 4;
  // two 4-element chunks per thread in flight; 16-byte accesses; r and d
  // are written once per pass (streaming stores)
  constexpr int UN = 2;
  const int64_t stride = (int64_t)nb * kThreads;
  for (int64_t k0 = (int64_t)lb * kThreads + threadIdx.x; k0 < n4; k0 += UN * stride) {
    V4<T> p[UN], q[UN], r[UN], d[UN];
    V4<double> u[UN];
#pragma unroll
    for (int c = 0; c < UN; ++c) {
      const int64_t k = k0 + c * stride;
      if (k < n4) {
        p[c] = ld4(a.p + 4 * k);
        q[c] = ld4(a.q + 4 * k);
        r[c] = ld4(a.r + 4 * k);
        if (a.d) d[c] = ld4(a.d + 4 * k);
        else u[c] = ld4(a.u + 4 * k);
      }
    }
#pragma unroll
    for (int c = 0; c < UN; ++c) {
      const int64_t k = k0 + c * stride;
      if (k < n4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          r[c].v[e] = r[c].v[e] - al * q[c].v[e];
          acc[0] += (double)r[c].v[e] * (double)r[c].v[e];
          acc[1] += (double)r[c].v[e];
          if (a.d) d[c].v[e] = d[c].v[e] + al * p[c].v[e];
          else u[c].v[e] += alpha * (double)p[c].v[e];
        }
        st4_nt(a.r + 4 * k, r[c]);
        if (a.d) st4_nt(a.d + 4 * k, d[c]);
        else st4(a.u + 4 * k, u[c]);
      }
    }
  }
  const int slots[2] = {PR_RR, PR_RSUM};
  write_partials<2>(a.st, slots, acc, lb);
  // a grid smaller than the residual stencil's leaves the rest of its
  // partial range at zero, so every consumer reads one count
  if (threadIdx.x == 0) {
    for (int k = lb + nb; k < a.nparts_out; k += nb) {
      part_row(a.st, PR_RR)[k] = 0.0;
      part_row(a.st, PR_RSUM)[k] = 0.0;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void axpy_kernel(AxpyArgs<T> a) {
  axpy_body<T>(a, (int)blockIdx.x, (int)gridDim.x);
}

// Grouped launch over a batch: each tile gets as many blocks as its stencil
// grid (so both producers of ||r||^2 write the same partial count).
template <class T>
__global__ __launch_bounds__(kThreads) void axpy_batched_kernel(const BatchTile<T>* tiles,
                                                                const int32_t* start, int ntiles,
                                                                int iter) {
  const int t = find_tile(start, ntiles, (int)blockIdx.x);
  const BatchTile<T>& bt = tiles[t];
  AxpyArgs<T> a;
  a.u = bt.U;
  a.r = bt.r;
  a.p = (iter & 1) ? bt.p1 : bt.p0;
  a.q = bt.q;
  a.n = bt.Np * bt.ld;
  a.nparts_pq = bt.st_nblk;
  a.iter = iter;
  a.st = bt.st;
  axpy_body<T>(a, (int)blockIdx.x - start[t], bt.st_nblk);
}

// ----------------------------------------------------------------------------
// Mean removal (last step of Algorithm 1): sum over the valid pixels, then
// subtract.  The padding stays zero.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void sum_kernel(const double* u, int64_t N, int64_t M,
                                                      int64_t ld, DevState st) {
  double acc[1] = {0.0};
  const int64_t n = N * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t j = k % ld;
    if (j < M) acc[0] += (double)u[k];
  }
  const int slots[1] = {PR_AUX};
  write_partials<1>(st, slots, acc, linear_block());
}

__global__ __launch_bounds__(kThreads) void sub_mean_kernel(double* u, int64_t N, int64_t M,
                                                           int64_t ld, DevState st,
                                                           int nparts) {
  const double s = reduce_slot(st, PR_AUX, nparts);
  const double mean = s / ((double)N * (double)M);
  if (blockIdx.x == 0 && threadIdx.x == 0) st.sc[SC_MEAN] = mean;
  const int64_t n = N * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t j = k % ld;
    if (j < M) u[k] -= mean;
  }
}

// End of a solve: u += d in FP64 (d, the solve's correction, in the vector
// type).
template <class T>
__global__ __launch_bounds__(kThreads) void commit_kernel(double* u, T* d, int64_t n4, int clear) {
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n4;
       k += (int64_t)gridDim.x * kThreads) {
    V4<double> x = ld4(u + 4 * k);
    const V4<T> c = ld4(d + 4 * k);
#pragma unroll
    for (int e = 0; e < 4; ++e) x.v[e] += (double)c.v[e];
    st4(u + 4 * k, x);
    if (clear) st4(d + 4 * k, zero4<T>());
  }
}

template <class T>
void launch_commit(double* u, T* d, int64_t n, hipStream_t s, bool clear) {
  hipLaunchKernelGGL(commit_kernel<T>, dim3(elementwise_blocks(n)), dim3(kThreads), 0, s, u, d,
                     n / 4, clear ? 1 : 0);
}
template void launch_commit<float>(double*, float*, int64_t, hipStream_t, bool);
template void launch_commit<double>(double*, double*, int64_t, hipStream_t, bool);

// ----------------------------------------------------------------------------
// Rounded output (Section 4, "rounded IRLS"): U made 2 pi-congruent to X.
// c = arg sum exp(i (X - U)) aligns the constant of U with X; then
// out = X + 2 pi rint((U + c - X) / 2 pi), every step in FP64 with explicit
// rounding so the integer decision is the one an FP64 evaluation takes.
// ----------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kThreads) void congruent_sum_kernel(const T* X, int64_t ldx,
                                                                const T* U, int64_t ldu, int64_t N,
                                                                int64_t M, DevState st) {
  double acc[2] = {0.0, 0.0};
  const int64_t n = N * M;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / M, j = k % M;
    const double d = __dsub_rn((double)X[i * ldx + j], (double)U[i * ldu + j]);
    double sn, cs;
    sincos(d, &sn, &cs);
    acc[0] += sn;
    acc[1] += cs;
  }
  const int slots[2] = {PT_A, PT_B};
  write_partials<2>(st, slots, acc, (int)blockIdx.x);
}

template <class T>
__global__ __launch_bounds__(kThreads) void congruent_apply_kernel(const T* X, int64_t ldx,
                                                                  const T* U, int64_t ldu, T* out,
                                                                  int64_t ldo, int64_t N, int64_t M,
                                                                  DevState st, int nparts) {
  const double sn = reduce_slot(st, PT_A, nparts);
  const double cs = reduce_slot(st, PT_B, nparts);
  const double c = atan2(sn, cs);
  const double two_pi = 6.283185307179586;
  const int64_t n = N * M;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / M, j = k % M;
    const double x = (double)X[i * ldx + j];
    const double t = __ddiv_rn(__dsub_rn(__dadd_rn((double)U[i * ldu + j], c), x), two_pi);
    out[i * ldo + j] = (T)__dadd_rn(x, __dmul_rn(two_pi, rint(t)));
  }
}

template <class T>
void launch_congruent(const T* X, int64_t ldx, const T* U, int64_t ldu, T* out, int64_t ldo,
                      int64_t N, int64_t M, DevState st, hipStream_t s) {
  const int nb = elementwise_blocks(N * M);
  hipLaunchKernelGGL(congruent_sum_kernel<T>, dim3(nb), dim3(kThreads), 0, s, X, ldx, U, ldu, N,
                     M, st);
  hipLaunchKernelGGL(congruent_apply_kernel<T>, dim3(nb), dim3(kThreads), 0, s, X, ldx, U, ldu,
                     out, ldo, N, M, st, nb);
}
template void launch_congruent<float>(const float*, int64_t, const float*, int64_t, float*,
                                      int64_t, int64_t, int64_t, DevState, hipStream_t);
template void launch_congruent<double>(const double*, int64_t, const double*, int64_t, double*,
                                       int64_t, int64_t, int64_t, DevState, hipStream_t);

// Copy the (mean-zero) internal U to the caller's N x M buffer.
template <class T>
__global__ __launch_bounds__(kThreads) void copy_out_kernel(const double* u, int64_t ld, T* out,
                                                           int64_t ldo, int64_t N, int64_t M) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (i < N && j < M) out[i * ldo + j] = (T)u[i * ld + j];
}

// Reduce the residual partials after a solve: ||r||^2 into SC_RR.
__global__ __launch_bounds__(kThreads) void finalize_rr_kernel(DevState st, int nparts) {
  const double rr = reduce_slot(st, PR_RR, nparts);
  if (threadIdx.x == 0) st.sc[SC_RR] = rr;
}

// Partial sums of squares of an array into the ||r||^2 slot (the step-level
// preconditioner of FP16 plans derives its input scale from them).
template <class T>
__global__ __launch_bounds__(kThreads) void sumsq_kernel(const T* x, int64_t n, DevState st) {
  double acc[1] = {0.0};
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads)
    acc[0] += (double)x[k] * (double)x[k];
  const int slots[1] = {PR_RR};
  write_partials<1>(st, slots, acc, linear_block());
}

template <class T>
int launch_sumsq(const T* x, int64_t n, DevState st, hipStream_t s) {
  const int nb = elementwise_blocks(n);
  hipLaunchKernelGGL(sumsq_kernel<T>, dim3(nb), dim3(kThreads), 0, s, x, n, st);
  return nb;
}
template int launch_sumsq<float>(const float*, int64_t, DevState, hipStream_t);

// Reduce one partial slot into a device double (step-level entry points).
__global__ __launch_bounds__(kThreads) void reduce_to_kernel(DevState st, int slot, int nparts,
                                                            double* out) {
  const double v = reduce_slot(st, slot, nparts);
  if (threadIdx.x == 0) *out = v;
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
template <class T>
void launch_setup(const SetupArgs<T>& a, hipStream_t s) {
  dim3 grid((unsigned)((a.ld + kThreads - 1) / kThreads), (unsigned)a.Np);
  hipLaunchKernelGGL(setup_kernel<T>, grid, dim3(kThreads), 0, s, a);
}

template <class T>
int launch_weights(const WeightsArgs<T>& a, hipStream_t s) {
  int rows = 1;
  const dim3 grid = weights_grid(a.Np, a.ld, &rows);
  hipLaunchKernelGGL(weights_kernel<T>, grid, dim3(kThreads), 0, s, a, rows);
  return (int)(grid.x * grid.y);
}

void launch_finalize_weights(DevState st, int nparts, double* out, double tol2, hipStream_t s,
                             int want_model) {
  hipLaunchKernelGGL(finalize_weights_kernel, dim3(1), dim3(kThreads), 0, s, st, nparts, out, tol2,
                     want_model);
}

// Weight-step grid: 256 columns per block, rows per block doubled until at
// most 2048 blocks (a batch reserves that many partial sums per tile).
dim3 weights_grid(int64_t Np, int64_t ld, int* rows_out) {
  const int64_t bx = (ld + kThreads - 1) / kThreads;
  int64_t rows = 1;
  while (bx * ((Np + rows - 1) / rows) > 2048) rows *= 2;
  *rows_out = (int)rows;
  return dim3((unsigned)bx, (unsigned)((Np + rows - 1) / rows));
}

int elementwise_blocks(int64_t n) {
  int64_t b = (n / 4 + kThreads - 1) / kThreads;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <class T>
int launch_axpy(const AxpyArgs<T>& a, hipStream_t s, int nblocks) {
  hipLaunchKernelGGL((axpy_kernel<T>), dim3(nblocks), dim3(kThreads), 0, s, a);
  return nblocks;
}

// Blocks of the CG update: one per compute unit of the 256, each streaming
// its share with two 16-byte chunks per array in flight per thread (512,
// 1024 and 2048 blocks measured slower at 8192^2), never more than the
// stencil's.
int axpy_blocks(int stencil_blocks) {
  return stencil_blocks < 256 ? stencil_blocks : 256;
}

void launch_mean_removal(double* u, int64_t N, int64_t M, int64_t ld, DevState st, hipStream_t s) {
  const int nb = elementwise_blocks(N * ld);
  hipLaunchKernelGGL(sum_kernel, dim3(nb), dim3(kThreads), 0, s, u, N, M, ld, st);
  hipLaunchKernelGGL(sub_mean_kernel, dim3(nb), dim3(kThreads), 0, s, u, N, M, ld, st, nb);
}

template <class T>
void launch_copy_out(const double* u, int64_t ld, T* out, int64_t ldo, int64_t N, int64_t M,
                     hipStream_t s) {
  dim3 grid((unsigned)((M + kThreads - 1) / kThreads), (unsigned)N);
  hipLaunchKernelGGL((copy_out_kernel<T>), grid, dim3(kThreads), 0, s, u, ld, out, ldo, N, M);
}

void launch_finalize_rr(DevState st, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(finalize_rr_kernel, dim3(1), dim3(kThreads), 0, s, st, nparts);
}

void launch_reduce_to(DevState st, int slot, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_to_kernel, dim3(1), dim3(kThreads), 0, s, st, slot, nparts, out);
}

template void launch_setup<float>(const SetupArgs<float>&, hipStream_t);
template void launch_setup<double>(const SetupArgs<double>&, hipStream_t);
template int launch_weights<float>(const WeightsArgs<float>&, hipStream_t);
template int launch_weights<double>(const WeightsArgs<double>&, hipStream_t);
template int launch_axpy<float>(const AxpyArgs<float>&, hipStream_t, int);

template <class T>
void launch_axpy_batched(const BatchTile<T>* tiles, const int32_t* start, int ntiles,
                         int total_blocks, int iter, hipStream_t s) {
  hipLaunchKernelGGL(axpy_batched_kernel<T>, dim3(total_blocks), dim3(kThreads), 0, s, tiles, start,
                     ntiles, iter);
}
template void launch_axpy_batched<float>(const BatchTile<float>*, const int32_t*, int, int, int,
                                         hipStream_t);
template int launch_axpy<double>(const AxpyArgs<double>&, hipStream_t, int);
template void launch_copy_out<float>(const double*, int64_t, float*, int64_t, int64_t, int64_t, hipStream_t);
template void launch_copy_out<double>(const double*, int64_t, double*, int64_t, int64_t, int64_t, hipStream_t);

}  // namespace irlsu
