// Folded preconditioner: the same z = P_N [(P_N^T r P_M) ./ (lambda + mu)] P_M^T
// (Section 3.3) at half the MFMA work, using the reflection symmetry of the
// DCT-II basis, P[n-1-i][k] = (-1)^k P[i][k] (n even, h = n/2):
//
//   forward   X[2k']   = sum_{i<h} (x[i] + x[n-1-i]) P[i][2k']
//             X[2k'+1] = sum_{i<h} (x[i] - x[n-1-i]) P[i][2k'+1]
//   inverse   E[i] = sum_k' P[i][2k'] X[2k'],  O[i] = sum_k' P[i][2k'+1] X[2k'+1]
//             x[i] = E[i] + O[i],  x[n-1-i] = E[i] - O[i]      (i < h)
//
// Each dense product becomes two independent h-wide products (the even and
// odd halves of the basis) on the same MFMA GEMM; cheap butterfly passes form
// the sums / differences before the forward products and recombine E, O
// after the inverse ones.  Spectral data are kept "even modes first".
#include <type_traits>

#include "kernels.hpp"

namespace irlsu {

// S[i][j'] = r[i][j] + r[i][M-1-j] (first half) / r[i][j] - r[i][M-1-j]
// (second half), j' = j < hM; zero padding; also used along the columns of
// the first intermediate (rows l', mirrored index i).
template <class TI, class TO>
__global__ __launch_bounds__(kThreads) void fold_rows_kernel(const TI* in, int64_t ldin, int64_t n,
                                                            int64_t rows_valid, int64_t rows,
                                                            TO* out, int64_t hp,
                                                            const double* dscale,
                                                            const int32_t* done) {
  if (done && *done) return;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= 2 * hp || i >= rows) return;
  using CT = typename std::conditional<sizeof(TO) == 8, double, float>::type;
  const CT scale = dscale ? (CT)*dscale : (CT)1;
  const int64_t h = n / 2;
  const int64_t half = c / hp, j = c % hp;
  CT v = 0;
  if (i < rows_valid && j < h) {
    const CT a = (CT)in[i * ldin + j];
    const CT b = (CT)in[i * ldin + (n - 1 - j)];
    v = (half == 0 ? a + b : a - b) * scale;
  }
  out[i * (2 * hp) + c] = (TO)v;
}

// T3[i][c] = E[i][c] + O[i][c] (i < hN), T3[N-1-i][c] = E[i][c] - O[i][c],
// with E rows [0, hNp) and O rows [hNp, 2 hNp) of the stacked input.
template <class OT>
__global__ __launch_bounds__(kThreads) void unfold_rows_kernel(const OT* eo, int64_t ld, int64_t N,
                                                              int64_t hNp, int64_t Np, OT* out,
                                                              const int32_t* done) {
  if (done && *done) return;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= ld || i >= Np) return;
  using CT = typename std::conditional<sizeof(OT) == 8, double, float>::type;
  const int64_t h = N / 2;
  CT v = 0;
  if (i < h) {
    v = (CT)eo[i * ld + c] + (CT)eo[(hNp + i) * ld + c];
  } else if (i < N) {
    const int64_t ii = N - 1 - i;
    v = (CT)eo[ii * ld + c] - (CT)eo[(hNp + ii) * ld + c];
  }
  out[i * ld + c] = (OT)v;
}

// z[i][j] = zE[i][j] + zO[i][j] (j < hM), z[i][M-1-j] = zE - zO, scaled;
// zero padding; FP64 partial sums z.r, z.q, sum z.
template <class T>
__global__ __launch_bounds__(kThreads) void unfold_cols_dots_kernel(const T* zeo, int64_t hMp,
                                                                   int64_t N, int64_t M, int64_t Np,
                                                                   int64_t ld, T* z, const T* r,
                                                                   const T* q, double zscale,
                                                                   const double* dscale,
                                                                   DevState st, int check_done) {
  if (check_done && st.fl[FL_DONE]) return;
  const double zs = dscale ? zscale / *dscale : zscale;
  const int64_t h = M / 2;
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t n = Np * ld;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads) {
    const int64_t i = k / ld, j = k % ld;
    double v = 0.0;
    if (i < N && j < M) {
      const T* row = zeo + i * (2 * hMp);
      if (j < h) v = (double)row[j] + (double)row[hMp + j];
      else {
        const int64_t jj = M - 1 - j;
        v = (double)row[jj] - (double)row[hMp + jj];
      }
      v *= zs;
    }
    const T zt = (T)v;
    z[k] = zt;
    const double zd = (double)zt;
    acc[0] += zd * (double)r[k];
    if (q) acc[1] += zd * (double)q[k];
    acc[2] += zd;
  }
  const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
  write_partials<3>(st, slots, acc, linear_block());
}

// Prologue of one application: convergence test on ||r||^2 (the first
// product's job in the dense form) and the FP16 input scale.
template <int NT>
__global__ __launch_bounds__(NT) void fold_prologue_kernel(DevState st, int nparts_rr,
                                                          int check_conv, int want_scale,
                                                          int64_t npix) {
  if (st.fl[FL_DONE]) return;
  const double rr = reduce_slot<NT>(st, PR_RR, nparts_rr);
  if (threadIdx.x != 0) return;
  if (check_conv) {
    st.sc[SC_RR] = rr;
    if (rr <= st.sc[SC_TOL2] * st.sc[SC_BB]) {
      st.fl[FL_DONE] = 1;
      return;
    }
  }
  // the same FP16 range argument as the dense form's first product
  // (want_scale < 0: the scale was set already, with the input it applies to)
  if (want_scale >= 0)
    st.sc[SC_SCALE] = want_scale ? (rr > 0.0 ? 1e-3 * sqrt((double)npix / rr) : 1.0) : 1.0;
}

void launch_fold_prologue(DevState st, int nparts_rr, int check_conv, int want_scale, int64_t npix,
                          hipStream_t s) {
  // one block; 1024 threads once there are many partials to read
  if (nparts_rr > 2048)
    hipLaunchKernelGGL(fold_prologue_kernel<1024>, dim3(1), dim3(1024), 0, s, st, nparts_rr,
                       check_conv, want_scale, npix);
  else
    hipLaunchKernelGGL(fold_prologue_kernel<kThreads>, dim3(1), dim3(kThreads), 0, s, st,
                       nparts_rr, check_conv, want_scale, npix);
}

// Folded basis tables of size n (even): Pe[i][k'] = P[i][2k'], Po[i][k'] =
// P[i][2k'+1] for i, k' < n/2 (hp x hp, zero padded) and their transposes;
// eig[k'] = lambda_{2k'}, eig[hp + k'] = lambda_{2k'+1} (+inf on padding).
template <class OT>
__global__ __launch_bounds__(kThreads) void fold_basis_kernel(int64_t n, int64_t hp, OT* Pe, OT* Pet,
                                                             OT* Po, OT* Pot, double* eig) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (k >= hp) return;
  const int64_t h = n / 2;
  double ve = 0.0, vo = 0.0;
  if (i < h && k < h) {
    const double c = sqrt(2.0 / (double)n);
    const int64_t ke = 2 * k, ko = 2 * k + 1;
    const double ae = 3.141592653589793 * (double)((ke * (2 * i + 1)) % (4 * n)) / (double)(2 * n);
    const double ao = 3.141592653589793 * (double)((ko * (2 * i + 1)) % (4 * n)) / (double)(2 * n);
    ve = cos(ae) * (ke == 0 ? sqrt(1.0 / (double)n) : c);
    vo = cos(ao) * c;
  }
  Pe[i * hp + k] = (OT)ve;
  Pet[k * hp + i] = (OT)ve;
  Po[i * hp + k] = (OT)vo;
  Pot[k * hp + i] = (OT)vo;
  if (i == 0) {
    if (k < h) {
      const double se = sin(3.141592653589793 * (double)(2 * k) / (double)(2 * n));
      const double so = sin(3.141592653589793 * (double)(2 * k + 1) / (double)(2 * n));
      eig[k] = 4.0 * se * se;
      eig[hp + k] = 4.0 * so * so;
    } else {
      eig[k] = __builtin_inf();
      eig[hp + k] = __builtin_inf();
    }
  }
}

void launch_fold_basis(int kind, int64_t n, int64_t hp, void* Pe, void* Pet, void* Po, void* Pot,
                       void* eig, hipStream_t s) {
  const dim3 grid((unsigned)((hp + kThreads - 1) / kThreads), (unsigned)hp);
  double* e = static_cast<double*>(eig);
  switch (kind) {
    case OK_F64:
      hipLaunchKernelGGL(fold_basis_kernel<double>, grid, dim3(kThreads), 0, s, n, hp,
                         static_cast<double*>(Pe), static_cast<double*>(Pet),
                         static_cast<double*>(Po), static_cast<double*>(Pot), e);
      break;
    case OK_F32:
      hipLaunchKernelGGL(fold_basis_kernel<float>, grid, dim3(kThreads), 0, s, n, hp,
                         static_cast<float*>(Pe), static_cast<float*>(Pet), static_cast<float*>(Po),
                         static_cast<float*>(Pot), e);
      break;
    case OK_BF16:
      hipLaunchKernelGGL(fold_basis_kernel<__bf16>, grid, dim3(kThreads), 0, s, n, hp,
                         static_cast<__bf16*>(Pe), static_cast<__bf16*>(Pet),
                         static_cast<__bf16*>(Po), static_cast<__bf16*>(Pot), e);
      break;
    case OK_F16:
      hipLaunchKernelGGL(fold_basis_kernel<_Float16>, grid, dim3(kThreads), 0, s, n, hp,
                         static_cast<_Float16*>(Pe), static_cast<_Float16*>(Pet),
                         static_cast<_Float16*>(Po), static_cast<_Float16*>(Pot), e);
      break;
  }
}

template <class TI, class TO>
void launch_fold_rows(const TI* in, int64_t ldin, int64_t n, int64_t rows_valid, int64_t rows,
                      TO* out, int64_t hp, const double* dscale, const int32_t* done,
                      hipStream_t s) {
  const dim3 grid((unsigned)((2 * hp + kThreads - 1) / kThreads), (unsigned)rows);
  hipLaunchKernelGGL((fold_rows_kernel<TI, TO>), grid, dim3(kThreads), 0, s, in, ldin, n,
                     rows_valid, rows, out, hp, dscale, done);
}

template <class OT>
void launch_unfold_rows(const OT* eo, int64_t ld, int64_t N, int64_t hNp, int64_t Np, OT* out,
                        const int32_t* done, hipStream_t s) {
  const dim3 grid((unsigned)((ld + kThreads - 1) / kThreads), (unsigned)Np);
  hipLaunchKernelGGL(unfold_rows_kernel<OT>, grid, dim3(kThreads), 0, s, eo, ld, N, hNp, Np, out,
                     done);
}

template <class T>
int launch_unfold_cols_dots(const T* zeo, int64_t hMp, int64_t N, int64_t M, int64_t Np, int64_t ld,
                            T* z, const T* r, const T* q, double zscale, const double* dscale,
                            DevState st, hipStream_t s) {
  const int nb = elementwise_blocks(Np * ld);
  hipLaunchKernelGGL(unfold_cols_dots_kernel<T>, dim3(nb), dim3(kThreads), 0, s, zeo, hMp, N, M, Np,
                     ld, z, r, q, zscale, dscale, st, 1);
  return nb;
}

#define FOLD_INST(TI, TO)                                                                        \
  template void launch_fold_rows<TI, TO>(const TI*, int64_t, int64_t, int64_t, int64_t, TO*,     \
                                         int64_t, const double*, const int32_t*, hipStream_t);
FOLD_INST(float, __bf16)
FOLD_INST(float, _Float16)
FOLD_INST(float, float)
FOLD_INST(double, double)
FOLD_INST(__bf16, __bf16)
FOLD_INST(_Float16, _Float16)
#undef FOLD_INST
template void launch_unfold_rows<__bf16>(const __bf16*, int64_t, int64_t, int64_t, int64_t, __bf16*,
                                         const int32_t*, hipStream_t);
template void launch_unfold_rows<_Float16>(const _Float16*, int64_t, int64_t, int64_t, int64_t,
                                           _Float16*, const int32_t*, hipStream_t);
template void launch_unfold_rows<float>(const float*, int64_t, int64_t, int64_t, int64_t, float*,
                                        const int32_t*, hipStream_t);
template void launch_unfold_rows<double>(const double*, int64_t, int64_t, int64_t, int64_t, double*,
                                         const int32_t*, hipStream_t);
template int launch_unfold_cols_dots<float>(const float*, int64_t, int64_t, int64_t, int64_t,
                                            int64_t, float*, const float*, const float*, double,
                                            const double*, DevState, hipStream_t);
template int launch_unfold_cols_dots<double>(const double*, int64_t, int64_t, int64_t, int64_t,
                                             int64_t, double*, const double*, const double*,
                                             double, const double*, DevState, hipStream_t);

}  // namespace irlsu
