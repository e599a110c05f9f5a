// Fast form of the preconditioner z = P_N [(P_N^T r P_M) ./ (lambda + mu)] P_M^T
// (Section 3.3; mode (0,0) set to zero, Appendix B) for power-of-two sides:
// the products with the orthonormal DCT-II basis are computed by fast
// cosine transforms instead of dense contractions, O(log n) work per pixel
// instead of O(n), which leaves the map bound by HBM traffic.
//
// One length-n DCT-II (n = 2h) of a row x:
//   v[m] = x[2m], v[n-1-m] = x[2m+1]          (even samples up, odd down)
//   w[m] = v[2m] + i v[2m+1]                  (v read as h complex numbers)
//   W = FFT_h(w)                              (Stockham radix-16/8/4/2 in LDS)
//   V_k = E_k + e^{-2 pi i k/n} O_k,  E_k = (W_k + conj W_{h-k}) / 2,
//                                      O_k = (W_k - conj W_{h-k}) / (2i)
//   c_k = e^{-i pi k/(2n)} V_k,  X_k = s_k Re c_k,  X_{n-k} = -s_{n-k} Im c_k
// with s_0 = sqrt(1/n), s_k = sqrt(2/n) (orthonormal).  The DCT-III (the
// transpose, i.e. the inverse) runs the same steps backwards, the inverse
// FFT as conj(FFT(conj(.))) / h.
//
// Passes of one application (FP32 arithmetic for FP32 and mixed plans, FP64
// for FP64 plans):
//   rows_fwd      T1[i][l]  = DCT-II along each row of r
//   transpose     T2 = T1^T
//   cols_fused    T1[l][.]  = DCT-III( DCT-II(T2[l][.]) ./ (lambda_k + mu_l) )
//   transpose     T2 = T1^T
//   rows_inv      z[i][.]   = DCT-III along each row of T2; z.r, z.q, sum z
// With plain beta (spectral path): cols also sums rhat^2 / (lambda + mu) =
// r.z (Parseval), a one-block kernel forms rho and beta, and rows_inv writes
// the direction p = z + beta p_old instead of z and its dots; the CG update
// r -= alpha q runs fused with rows_fwd of the next application
// (fct_rows_fwd_cg_kernel, alpha from cg_alpha_kernel) and d += alpha p with
// rows_inv, which reads p_old anyway.  Sides that are not powers of two run
// the same passes with run-time sizes (fctg.hip).
#include <type_traits>

#include "fft.hpp"
#include "kernels.hpp"

namespace irlsu {

// ---- Stockham FFT of ROWS rows of H complex points held in LDS ----------
// LDS holds complex point x at slot pc(x) = x + x / 16: one pad slot per 16
// points keeps the stride-16 writes of the first stages (and the strided
// reads of the last) off a single bank.
__device__ __forceinline__ int pc(int x) { return x + (x >> 4); }
template <int NPTS>
constexpr int padded() {
  return NPTS + NPTS / 16;
}
// real element e of the block's rows (two per complex slot)
__device__ __forceinline__ int pr(int e) { return 2 * pc(e >> 1) + (e & 1); }

// Twiddles of the stage with span NS and radix R, from its table: entry
// (NS - 1) + (r - 1) NS + k holds e^{-2 pi i r k / (NS R)}, r = 1..R-1,
// k = 0..NS-1 (the stages' tables end to end fill h - 1 entries).  Each
// value is rounded once from FP64, and a load replaces the products that
// would form it.
//
// w, w^2, w^4, w^8 come from the table and the others as products of two of
// them (at most three roundings).  Loading every power from the global table
// instead was measured slower in all three passes at 8192^2 (more loads per
// stage, whose waits also wait for the pass's own earlier loads).  The
// column pass, bound by instruction issue, reads every power of its span-16
// stage from a block-local copy of that stage's table in LDS (LT16 below).
template <class CT, int R, int NS>
__device__ __forceinline__ void stage_twiddles(const Cx<CT>* __restrict__ tw, int k,
                                               Cx<CT> (&w)[R]) {
  const Cx<CT>* t = tw + (NS - 1) + k;
  w[1] = t[0];
  if constexpr (R > 2) {
    w[2] = t[NS];
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (R > 4) {
    w[4] = t[3 * NS];
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  }
  if constexpr (R > 8) {
    w[8] = t[7 * NS];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
  }
}

// Entries of the span-16 stage's table (radix min(16, H / 16)); 0 when the
// transform has no such stage.
template <int H>
constexpr int lt16_size() {
  return H >= 32 ? ((H / 16 >= 16 ? 16 : H / 16) - 1) * 16 : 0;
}

// Stage with span NS and radix R: butterfly j of a row reads points
// j + r H/R, applies e^{-2 pi i r (j mod NS) / (NS R)}, and writes the
// R-point DFT to (j / NS) NS R + (j mod NS) + r NS.  In place: every thread
// holds its butterflies in registers across a barrier.  With the one-slot
// pad per 16 points, the R points of a butterfly sit at constant offsets
// from the first one (H/R and NS multiples of 16, or NS = 1 with R = 16
// and the first point on a multiple of 16), so one address serves all R.
// LT16: the span-16 stage reads its twiddles from lt16, the LDS copy of
// its table (entry (r - 1) 16 + k).
template <class CT, int H, int ROWS, int R, int NS, bool LT16>
__device__ __forceinline__ void fft_stage(Cx<CT>* buf, const Cx<CT>* __restrict__ tw,
                                          const Cx<CT>* lt16, int tid) {
  constexpr int BPR = H / R;
  constexpr int NB = ROWS * BPR / kThreads;
  static_assert(NB >= 1 && NB * kThreads == ROWS * BPR, "butterflies per thread");
  constexpr bool RD_CONST = BPR % 16 == 0;
  constexpr int RD_STRIDE = BPR + BPR / 16;
  constexpr bool WR_CONST = NS % 16 == 0 || (NS == 1 && R == 16);
  constexpr int WR_STRIDE = NS == 1 ? 1 : NS + NS / 16;
  Cx<CT> a[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int bi = tid + b * kThreads;
    const int row = bi / BPR, j = bi % BPR;
    const int k = j % NS;
    const int src = row * H + j;
    if constexpr (RD_CONST) {
      const Cx<CT>* sp = buf + pc(src);
#pragma unroll
      for (int r = 0; r < R; ++r) a[b][r] = sp[r * RD_STRIDE];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) a[b][r] = buf[pc(src + r * BPR)];
    }
    if constexpr (NS > 1) {
      Cx<CT> w[R];
      if constexpr (LT16 && NS == 16) {
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = lt16[(r - 1) * 16 + k];
      } else {
        stage_twiddles<CT, R, NS>(tw, k, w);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) a[b][r] = cmul(a[b][r], w[r]);
    }
    dft<CT, R>(a[b]);
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int bi = tid + b * kThreads;
    const int row = bi / BPR, j = bi % BPR;
    const int k = j % NS;
    const int dst = row * H + (j / NS) * NS * R + k;
    if constexpr (WR_CONST) {
      Cx<CT>* dp = buf + pc(dst);
#pragma unroll
      for (int r = 0; r < R; ++r) dp[r * WR_STRIDE] = a[b][r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pc(dst + r * NS)] = a[b][r];
    }
  }
  __syncthreads();
}

template <class CT, int H, int ROWS, bool LT16, int NS = 1>
__device__ __forceinline__ void fft_rows(Cx<CT>* buf, const Cx<CT>* __restrict__ tw, int tid,
                                         const Cx<CT>* lt16 = nullptr) {
  if constexpr (NS < H) {
    constexpr int REM = H / NS;
    constexpr int R = REM >= 16 ? 16 : REM;
    fft_stage<CT, H, ROWS, R, NS, LT16>(buf, tw, lt16, tid);
    fft_rows<CT, H, ROWS, LT16, NS * R>(buf, tw, tid, lt16);
  }
}

// Rows per block: at least 4096 complex points per block so that every
// stage has one butterfly per thread or more.
template <int H>
constexpr int rows_per_block() {
  return H >= 4096 ? 1 : 4096 / H;
}

// Tables of one side n = 2h (CT): complex [0, h - 1) the FFT stages'
// twiddles (stage_twiddles), entry h - 1 unused; [h, 2h] e^{-2 pi i k/n},
// k = 0..h; [2h+1, 3h+1] e^{-i pi k/(2n)}, k = 0..h; then the h/2 + 1
// records of the column pass's pair steps (PairTw), whose eigenvalues 4
// sin^2(pi k / 2n) of the side's Neumann second difference are stored times
// 2n (a power of two: 1 / (2n lambda + 2n mu) is the division and the
// inverse transform's output scale 1/(4h) at once, with the same roundings).
template <class CT>
struct Tw {
  const Cx<CT>* fft;
  const Cx<CT>* tn;
  const Cx<CT>* tq;
  const PairTw<CT>* pair;
};
template <class CT, int H>
__device__ __forceinline__ Tw<CT> tw_of(const void* p) {
  const Cx<CT>* t = static_cast<const Cx<CT>*>(p);
  return {t, t + H, t + 2 * H + 1,
          reinterpret_cast<const PairTw<CT>*>(static_cast<const CT*>(p) +
                                               pair_table_offset(H))};
}

// position of row element e in the even-up / odd-down sequence v
template <int N>
__device__ __forceinline__ int perm(int e) {
  return (e & 1) ? N - 1 - (e >> 1) : (e >> 1);
}

// Pair steps of one row held in LDS (post_core and pre_core), the twiddles
// from the side's tables.  post_pair returns twice the coefficients: the
// even/odd split's factor 1/2 is left to the caller's own scale (a power of
// two, so every rounding is unchanged); so does pre_pair.
template <class CT, int H>
__device__ __forceinline__ void post_pair(const Cx<CT>* buf, int base, int k, const Tw<CT>& tw,
                                          Cx<CT>& ck, Cx<CT>& cp) {
  post_core(buf[pc(base + (k & (H - 1)))], buf[pc(base + ((H - k) & (H - 1)))], tw.tq[k],
            tw.tq[H - k], tw.tn[k], ck, cp);
}

template <class CT, int H>
__device__ __forceinline__ void pre_pair(Cx<CT> ck, Cx<CT> cp, int k, const Tw<CT>& tw, Cx<CT>* buf,
                                         int base) {
  Cx<CT> sk, sp;
  pre_core(ck, cp, tw.tq[k], tw.tq[H - k], tw.tn[k], sk, sp);
  buf[pc(base + (k & (H - 1)))] = sk;
  if (k != H - k && k > 0) buf[pc(base + H - k)] = sp;
}

// ---- row staging ----------------------------------------------------------
// Every thread moves whole 16-byte chunks of the block's rows; all of a
// thread's global loads are issued before its first LDS write.
template <class TI, int H>
struct RowChunks {
  static constexpr int N = 2 * H, ROWS = rows_per_block<H>();
  static constexpr int W = Vec16<TI>::W;
  static constexpr int NCH = ROWS * N / W / kThreads;
  static_assert(NCH * W * kThreads == ROWS * N, "chunks per thread");
  typename Vec16<TI>::type d[NCH];
};

// registers <- the block's rows row0 .. row0 + ROWS - 1 (natural order)
template <class TI, int H>
__device__ __forceinline__ void load_rows(const TI* __restrict__ in, int64_t ld, int64_t row0,
                                          RowChunks<TI, H>& ch, int tid) {
  using RC = RowChunks<TI, H>;
  using V = typename Vec16<TI>::type;
#pragma unroll
  for (int i = 0; i < RC::NCH; ++i) {
    const int e0 = (tid + i * kThreads) * RC::W;
    const int row = e0 / RC::N, c = e0 % RC::N;
    ch.d[i] = ld_nt<V>(in + (row0 + row) * ld + c);
  }
}

// LDS <- registers, in the even-up / odd-down order, as CT times scale
template <class CT, class TI, int H>
__device__ __forceinline__ void put_rows(const RowChunks<TI, H>& ch, CT* v, CT scale, int tid) {
  using RC = RowChunks<TI, H>;
  constexpr int N = RC::N, W = RC::W;
#pragma unroll
  for (int i = 0; i < RC::NCH; ++i) {
    const int e0 = (tid + i * kThreads) * W;
    const int row = e0 / N, c = e0 % N;
    if constexpr (W >= 4) {
      // a chunk of W elements at c (a multiple of W) fills W / 4 complex
      // slots from the front (even elements, c/4 + s) and W / 4 from the back
      // (odd ones, h - 1 - c/4 - s), two elements each
      Cx<CT>* b = reinterpret_cast<Cx<CT>*>(v);
#pragma unroll
      for (int s4 = 0; s4 < W / 4; ++s4) {
        b[pc(row * H + c / 4 + s4)] = {(CT)ch.d[i][4 * s4] * scale,
                                       (CT)ch.d[i][4 * s4 + 2] * scale};
        b[pc(row * H + H - 1 - c / 4 - s4)] = {(CT)ch.d[i][4 * s4 + 3] * scale,
                                               (CT)ch.d[i][4 * s4 + 1] * scale};
      }
    } else {
#pragma unroll
      for (int t = 0; t < W; ++t) v[pr(row * N + perm<N>(c + t))] = (CT)ch.d[i][t] * scale;
    }
  }
}

// LDS <- registers for the inverse pre-processing: element e of a row goes
// to complex slot e (real part) for e < h and to slot (n - e) mod h
// (imaginary part) for e >= h, so that slot k holds (x_k, x_{n-k}) and slot
// h - k holds (x_{h-k}, x_{h+k}) -- the four inputs of pair k sit in the two
// slots that pair k overwrites (slot 0 holds (x_0, x_h)).
template <class CT, class TI, int H>
__device__ __forceinline__ void put_rows_inv(const RowChunks<TI, H>& ch, Cx<CT>* buf, int tid) {
  using RC = RowChunks<TI, H>;
  constexpr int N = RC::N;
  CT* v = reinterpret_cast<CT*>(buf);
#pragma unroll
  for (int i = 0; i < RC::NCH; ++i) {
    const int e0 = (tid + i * kThreads) * RC::W;
    const int row = e0 / N, c = e0 % N;
#pragma unroll
    for (int t = 0; t < RC::W; ++t) {
      const int e = c + t;
      const int slot = e < H ? e : (N - e) & (H - 1);
      v[2 * pc(row * H + slot) + (e < H ? 0 : 1)] = (CT)ch.d[i][t];
    }
  }
}

// W output elements at c (a multiple of W, W >= 4) of a row after the
// inverse FFT, the inverse of put_rows' slot map:
// w = conj(FFT(conj W)) / h, so odd positions take the negated imaginary part
template <class CT, int H, int W, class OT>
__device__ __forceinline__ void inv_chunk(const Cx<CT>* buf, int row, int c, CT inv_h,
                                          OT (&o)[W]) {
  static_assert(W >= 4 && W % 4 == 0, "chunk");
#pragma unroll
  for (int s4 = 0; s4 < W / 4; ++s4) {
    const Cx<CT> A = buf[pc(row * H + c / 4 + s4)];
    const Cx<CT> B = buf[pc(row * H + H - 1 - c / 4 - s4)];
    o[4 * s4] = (OT)(A.x * inv_h);
    o[4 * s4 + 1] = (OT)(-B.y * inv_h);
    o[4 * s4 + 2] = (OT)(-A.y * inv_h);
    o[4 * s4 + 3] = (OT)(B.x * inv_h);
  }
}

// value of output element c of a row after the inverse FFT:
// w = conj(FFT(conj W)) / h, v[2m] = Re w[m], v[2m+1] = Im w[m]
template <class CT, int N>
__device__ __forceinline__ CT inv_value(const CT* v, int row, int c, CT inv_h) {
  const int m = perm<N>(c);
  const CT x = v[pr(row * N + m)];
  return ((m & 1) ? -x : x) * inv_h;
}

// ---- pass 1: DCT-II along rows ------------------------------------------
template <class CT, class TI, class TO, int H>
__global__ __launch_bounds__(kThreads) void fct_rows_fwd_kernel(const TI* __restrict__ in,
                                                               int64_t ld, TO* __restrict__ out,
                                                               const void* twp,
                                                               const int32_t* done,
                                                               const double* dscale) {
  if (*done) return;
  constexpr int N = 2 * H, ROWS = rows_per_block<H>();
  constexpr int NP = H / 2 + 1;
  constexpr int PP = (ROWS * NP + kThreads - 1) / kThreads;
  __shared__ Cx<CT> buf[padded<ROWS * H>()];
  const Tw<CT> tw = tw_of<CT, H>(twp);
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  CT* v = reinterpret_cast<CT*>(buf);
  {
    RowChunks<TI, H> ch;
    load_rows<TI, H>(in, ld, row0, ch, tid);
    put_rows<CT, TI, H>(ch, v, dscale ? (CT)*dscale : (CT)1, tid);
  }
  __syncthreads();
  fft_rows<CT, H, ROWS, false>(buf, tw.fft, tid);
  // s_k / 2: post_pair returns twice the coefficient
  const CT s0 = (CT)(0.5 * sqrt(1.0 / N)), s1 = (CT)(0.5 * sqrt(2.0 / N));
#pragma unroll
  for (int qq = 0; qq < PP; ++qq) {
    const int p = tid + qq * kThreads;
    if (p < ROWS * NP) {
      const int row = ROWS == 1 ? 0 : p / NP, k = ROWS == 1 ? p : p % NP;
      Cx<CT> ck, cp;
      post_pair<CT, H>(buf, row * H, k, tw, ck, cp);
      TO* o = out + (row0 + row) * ld;
      o[k] = (TO)(ck.x * (k == 0 ? s0 : s1));
      if (k > 0) o[N - k] = (TO)(-ck.y * s1);
      if (H - k != k) {
        o[H - k] = (TO)(cp.x * s1);
        if (k > 0) o[H + k] = (TO)(-cp.y * s1);
      }
    }
  }
}

// ---- CG update fused with pass 1 ---------------------------------------
// alpha = rho / p.q (p.q and ||q||^2 from the stencil's partials); the FP16
// input scale of the next application from the bound ||r - alpha q|| <=
// ||r|| + |alpha| ||q|| (||r||^2 as the last convergence test stored it), so
// the new residual's scaled values stay at or below the usual 1e-3 rms.
__global__ __launch_bounds__(1024) void cg_alpha_kernel(DevState st, int nparts_pq, int iter,
                                                       int f16, double npix) {
  if (st.fl[FL_DONE]) return;
  const double pq = reduce_slot<1024>(st, PR_PQ, nparts_pq);
  const double qq = reduce_slot<1024>(st, PR_AUX, nparts_pq);
  if (threadIdx.x != 0) return;
  const double rho = st.sc[SC_RHO + (iter & 1)];
  if (!(pq > 0.0) || !(rho >= 0.0) || !isfinite(pq)) {
    st.fl[FL_STATUS] |= 1;
    st.fl[FL_DONE] = 1;
    return;
  }
  const double alpha = rho / pq;
  st.sc[SC_ALPHA + (iter & 1)] = alpha;
  st.sc[SC_PQ] = pq;
  st.fl[FL_ITERS] += 1;  // counted on the device: iteration-independent launches
  if (f16) {
    const double bound = sqrt(st.sc[SC_RR]) + fabs(alpha) * sqrt(qq);
    st.sc[SC_SCALE] = bound > 0.0 ? 1e-3 * sqrt(npix) / bound : 1.0;
  }
}

// Per row group: r -= alpha q (written back, streaming), the new r (times
// the input scale) transformed like pass 1 into out; partials ||r||^2 and
// sum r, zero padded to nparts_out.  (d += alpha p waits for the row DCT-III
// pass, which reads p for the next direction: 12 bytes per pixel less here
// for 8 more there.)
template <class CT, class T, class TO, int H>
__global__ __launch_bounds__(kThreads) void fct_rows_fwd_cg_kernel(
    T* __restrict__ r, const T* __restrict__ q, int64_t ld, TO* __restrict__ out,
    const void* twp, DevState st, int iter, int f16, int nparts_out) {
  if (st.fl[FL_DONE]) return;
  constexpr int N = 2 * H, ROWS = rows_per_block<H>();
  constexpr int NP = H / 2 + 1;
  constexpr int PP = (ROWS * NP + kThreads - 1) / kThreads;
  using RC = RowChunks<T, H>;
  using V = typename Vec16<T>::type;
  constexpr int W = RC::W;
  __shared__ Cx<CT> buf[padded<ROWS * H>()];
  const Tw<CT> tw = tw_of<CT, H>(twp);
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  CT* v = reinterpret_cast<CT*>(buf);
  const T al = (T)st.sc[SC_ALPHA + (iter & 1)];
  double acc[2] = {0.0, 0.0};
  {
    RC ch;
    constexpr int UN = RC::NCH < 2 ? RC::NCH : 2;
#pragma unroll
    for (int i0 = 0; i0 < RC::NCH; i0 += UN) {
      V qv[UN], rv[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int e0 = (tid + (i0 + u) * kThreads) * W;
        const int64_t o = (row0 + e0 / N) * ld + e0 % N;
        qv[u] = ld_nt<V>(q + o);
        rv[u] = ld_nt<V>(r + o);
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int e0 = (tid + (i0 + u) * kThreads) * W;
        const int64_t o = (row0 + e0 / N) * ld + e0 % N;
#pragma unroll
        for (int t = 0; t < W; ++t) {
          rv[u][t] = rv[u][t] - al * qv[u][t];
          acc[0] += (double)rv[u][t] * (double)rv[u][t];
          acc[1] += (double)rv[u][t];
        }
        __builtin_nontemporal_store(rv[u], reinterpret_cast<V*>(r + o));
        ch.d[i0 + u] = rv[u];
      }
    }
    put_rows<CT, T, H>(ch, v, f16 ? (CT)st.sc[SC_SCALE] : (CT)1, tid);
  }
  __syncthreads();
  fft_rows<CT, H, ROWS, false>(buf, tw.fft, tid);
  // s_k / 2: post_pair returns twice the coefficient
  const CT s0 = (CT)(0.5 * sqrt(1.0 / N)), s1 = (CT)(0.5 * sqrt(2.0 / N));
#pragma unroll
  for (int qq = 0; qq < PP; ++qq) {
    const int pp = tid + qq * kThreads;
    if (pp < ROWS * NP) {
      const int row = ROWS == 1 ? 0 : pp / NP, k = ROWS == 1 ? pp : pp % NP;
      Cx<CT> ck, cp;
      post_pair<CT, H>(buf, row * H, k, tw, ck, cp);
      TO* o = out + (row0 + row) * ld;
      o[k] = (TO)(ck.x * (k == 0 ? s0 : s1));
      if (k > 0) o[N - k] = (TO)(-ck.y * s1);
      if (H - k != k) {
        o[H - k] = (TO)(cp.x * s1);
        if (k > 0) o[H + k] = (TO)(-cp.y * s1);
      }
    }
  }
  const int slots[2] = {PR_RR, PR_RSUM};
  write_partials<2>(st, slots, acc, (int)blockIdx.x);
  if (threadIdx.x == 0) {
    for (int k = (int)blockIdx.x + (int)gridDim.x; k < nparts_out; k += (int)gridDim.x) {
      part_row(st, PR_RR)[k] = 0.0;
      part_row(st, PR_RSUM)[k] = 0.0;
    }
  }
}

// ---- pass 3: DCT-II, spectral division, DCT-III along rows of the
// transposed intermediate (the columns of the image) ----------------------
template <class CT, class ST, int H, bool RHO>
__global__ __launch_bounds__(kThreads) void fct_cols_kernel(ST* __restrict__ io, int64_t ld,
                                                           const void* twp,
                                                           const double* __restrict__ eig_l,
                                                           DevState st) {
  if (st.fl[FL_DONE]) return;
  constexpr int N = 2 * H, ROWS = rows_per_block<H>();
  constexpr int NP = H / 2 + 1;
  constexpr int PP = (ROWS * NP + kThreads - 1) / kThreads;
  constexpr int NT16 = lt16_size<H>();
  constexpr bool LT16 = NT16 > 0;
  __shared__ Cx<CT> buf[padded<ROWS * H>()];
  __shared__ Cx<CT> lt16[LT16 ? NT16 : 1];
  const Tw<CT> tw = tw_of<CT, H>(twp);
  const int tid = threadIdx.x;
  if constexpr (LT16) {
    static_assert(NT16 <= kThreads, "one table entry per thread");
    if (tid < NT16) lt16[tid] = tw.fft[15 + tid];
  }
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  CT* v = reinterpret_cast<CT*>(buf);
  // RHO: this thread's share of sum rhat^2 / (lambda + mu), in units of
  // (2 c)^2 s_k^2 / 2 -- see the scale at the end
  CT rho = (CT)0;
  {
    RowChunks<ST, H> ch;
    load_rows<ST, H>(io, ld, row0, ch, tid);
    put_rows<CT, ST, H>(ch, v, (CT)1, tid);
  }
  __syncthreads();
  fft_rows<CT, H, ROWS, LT16>(buf, tw.fft, tid, lt16);
  // mu times 2n, as the pair records' eigenvalues (exact)
  const CT mu0 = (CT)(eig_l[row0] * (2.0 * N));
  // forward post-processing, division and inverse pre-processing of pair
  // (k, h-k), in place: the pair's two slots are read and written by the
  // same thread only.  With d = 1 / (lambda_k + mu_l), the scaled
  // coefficient divided by s_k is Re(c_k) d_k, and -Im(c_k) d_{n-k} at n-k
  // (here all of them twice over, from post_core, and twice again from
  // pre_core: with the inverse FFT's 1/h, an output scale of 1/(4h) = 1/(2n),
  // which d takes along).
#pragma unroll
  for (int qq = 0; qq < PP; ++qq) {
    const int p = tid + qq * kThreads;
    if (p < ROWS * NP) {
      const int row = ROWS == 1 ? 0 : p / NP, k = ROWS == 1 ? p : p % NP;
      const int64_t l = row0 + row;
      const CT mu = ROWS == 1 ? mu0 : (CT)(eig_l[l] * (2.0 * N));
      // one aligned record holds the pair's twiddles and eigenvalues
      const PairTw<CT> pt = tw.pair[k];
      Cx<CT>* slot_k = buf + pc(row * H + (k & (H - 1)));
      Cx<CT>* slot_p = buf + pc(row * H + ((H - k) & (H - 1)));
      Cx<CT> ck, cp;
      post_core(*slot_k, *slot_p, pt.q, pt.qp, pt.n, ck, cp);
      // d = 1 / (lambda + mu) / (2n) at k, n-k, h-k, h+k (mode (0, 0) set
      // to zero)
      const CT dk = (l == 0 && k == 0) ? (CT)0 : recip(pt.e[0] + mu);
      const CT dnk = k > 0 ? recip(pt.e[1] + mu) : (CT)0;
      const CT dp = recip(pt.e[2] + mu), dnp = recip(pt.e[3] + mu);
      // X~ at k, n-k, h-k, h+k; c_k (inverse) = X~_k - i X~_{n-k}
      const CT xk = ck.x * dk;
      const CT xnk = k > 0 ? -ck.y * dnk : (CT)0;
      const CT xp = cp.x * dp;
      const CT xnp = -cp.y * dnp;   // k = 0: index h, equal to xp
      Cx<CT> sk, sp;
      pre_core<CT>({xk, -xnk}, {xp, -xnp}, pt.q, pt.qp, pt.n, sk, sp);
      *slot_k = sk;
      if (k != H - k && k > 0) *slot_p = sp;
      if constexpr (RHO) {
        // squared orthonormal coefficients (s_k Re c_k etc.) over the
        // eigenvalue sum; each index of the column once (k = 0 and k = h/2
        // hold two of them, not four).  s_0^2 = 1/n is half of the other
        // s_k^2 = 2/n, which the scale at the end carries.
        rho += (k == 0 ? (CT)0.5 : (CT)1) * ck.x * ck.x * dk;
        if (k > 0) rho += ck.y * ck.y * dnk;
        if (k < H / 2) rho += cp.x * cp.x * dp;
        if (k > 0 && k < H / 2) rho += cp.y * cp.y * dnp;
      }
    }
  }
  __syncthreads();
  fft_rows<CT, H, ROWS, LT16>(buf, tw.fft, tid, lt16);
  // the output scale 1/(4h) came with d
  const CT inv_h = (CT)1;
  using V = typename Vec16<ST>::type;
  constexpr int W = Vec16<ST>::W;
  constexpr int NCH = ROWS * N / W / kThreads;
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    const int e0 = (tid + i * kThreads) * W;
    const int row = e0 / N, c = e0 % N;
    V o;
    if constexpr (W >= 4) {
      ST ot[W];
      inv_chunk<CT, H, W, ST>(buf, row, c, inv_h, ot);
#pragma unroll
      for (int t = 0; t < W; ++t) o[t] = ot[t];
    } else {
#pragma unroll
      for (int t = 0; t < W; ++t) o[t] = (ST)inv_value<CT, N>(v, row, c + t, inv_h);
    }
    *reinterpret_cast<V*>(io + (row0 + row) * ld + c) = o;
  }
  if constexpr (RHO) {
    // (2 c)^2 -> c^2 and the factor s_k^2 = 2/n: 1/(2n), which d carried
    double acc[1] = {(double)rho};
    const int slots[1] = {PR_ZR};
    write_partials<1>(st, slots, acc, (int)blockIdx.x);
  }
}

// rho = sum of the column pass's partials (divided by the square of the FP16
// input scale), stored for iteration iter with beta = rho / rho_{iter-1}
// (0 at iter 0).  nparts_rr > 0: also the convergence test on the ||r||^2
// partials of the fused update (the prologue's job on the other path; a
// converged solve then wasted only the passes before this one).  Run by the
// first block of the transpose that follows the column pass.
template <int NT>
__device__ __forceinline__ void rho_body(const DevState& st, int n, int iter, int f16,
                                         int nparts_rr) {
  double rho = reduce_slot<NT>(st, PR_ZR, n);
  const double rr = nparts_rr > 0 ? reduce_slot<NT>(st, PR_RR, nparts_rr) : 0.0;
  if (threadIdx.x == 0) {
    if (nparts_rr > 0) {
      st.sc[SC_RR] = rr;
      if (rr <= st.sc[SC_TOL2] * st.sc[SC_BB]) {
        st.fl[FL_DONE] = 1;
        st.fl[FL_DPEND] = 1;   // d += alpha p of this iteration is still owed
        return;
      }
    }
    if (f16) {
      const double sc = st.sc[SC_SCALE];
      rho /= sc * sc;
    }
    st.sc[SC_RHO + (iter & 1)] = rho;
    st.sc[SC_BETA] = iter > 0 ? rho / st.sc[SC_RHO + ((iter - 1) & 1)] : 0.0;
  }
}


// ---- pass 5: DCT-III along rows, z.r, z.q, sum z -------------------------
// The stored coefficients go to LDS by put_rows_inv, so that each pair's four
// inputs sit in the two slots the pair overwrites: the pre-processing runs in
// place with no barrier between its reads and writes.
// OUT: 0 z and the dots z.r, sum z; 1 also z.q (flexible beta); 2 the new
// direction p = z + beta p_in into z (p_in, passed as q, unread at iter 0),
// no dots, and with dacc non-null the iterate update of the iteration
// before, dacc += alpha_{iter-1} p_in -- alone if the rho step stopped the
// solve on convergence (FL_DPEND).
template <class CT, class SI, class TO, int H, int OUT>
__global__ __launch_bounds__(kThreads) void fct_rows_inv_kernel(
    const SI* __restrict__ in, int64_t ld, TO* __restrict__ z, const TO* __restrict__ r,
    const TO* __restrict__ q, TO* __restrict__ dacc, const void* twp, DevState st,
    int use_scale, int iter) {
  constexpr bool FLEX = OUT == 1;
  constexpr int N = 2 * H, ROWS = rows_per_block<H>();
  using V = typename Vec16<TO>::type;
  constexpr int W = Vec16<TO>::W;
  constexpr int NCH = ROWS * N / W / kThreads;
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  const bool dupd = OUT == 2 && dacc != nullptr && iter != 0;
  const TO al = dupd ? (TO)st.sc[SC_ALPHA + ((iter - 1) & 1)] : (TO)0;
  // chunk b of this thread: dacc += alpha p_in
  auto add_dir = [&](int b, const V& pb) {
    const int e0 = (tid + b * kThreads) * W;
    TO* dp = dacc + (row0 + e0 / N) * ld + e0 % N;
    V dv = ld_nt<V>(dp);
#pragma unroll
    for (int t = 0; t < W; ++t) dv[t] = dv[t] + al * pb[t];
    st_nt<V>(dp, dv);
  };
  if (st.fl[FL_DONE]) {
    if (dupd && st.fl[FL_DPEND]) {
#pragma unroll
      for (int b = 0; b < NCH; ++b) {
        const int e0 = (tid + b * kThreads) * W;
        add_dir(b, ld_nt<V>(q + (row0 + e0 / N) * ld + e0 % N));
      }
    }
    return;
  }
  constexpr int NP = H / 2 + 1;
  constexpr int PP = (ROWS * NP + kThreads - 1) / kThreads;
  __shared__ Cx<CT> buf[padded<ROWS * H>()];
  const Tw<CT> tw = tw_of<CT, H>(twp);
  CT* v = reinterpret_cast<CT*>(buf);
  // output scale: 1/h of the inverse FFT and the 1/2 that pre_pair leaves
  // out, undoing the input scale of the first pass when the intermediates
  // are FP16
  const CT inv_h = (CT)(0.5 / H) / (use_scale ? (CT)st.sc[SC_SCALE] : (CT)1);
  const CT is0 = (CT)sqrt((double)N), is1 = (CT)sqrt(0.5 * N);   // 1 / s_k
  // OUT 2: the previous direction, loaded with the stored coefficients so
  // that its latency hides behind the transform (NCH 16-byte chunks per
  // thread, 8 at h = 4096 in FP32; rows longer than that load it after the
  // transform instead, to keep the registers for the butterflies)
  constexpr bool PRE = OUT == 2 && NCH <= 8;
  constexpr int NPV = OUT == 2 ? NCH : 1;
  V pv[NPV];
  {
    RowChunks<SI, H> ch;
    load_rows<SI, H>(in, ld, row0, ch, tid);
    if constexpr (PRE) {
      if (iter != 0) {
#pragma unroll
        for (int b = 0; b < NCH; ++b) {
          const int e0 = (tid + b * kThreads) * W;
          pv[b] = ld_nt<V>(q + (row0 + e0 / N) * ld + e0 % N);
        }
        if (dupd) {
#pragma unroll
          for (int b = 0; b < NCH; ++b) add_dir(b, pv[b]);
        }
      }
    }
    put_rows_inv<CT, SI, H>(ch, buf, tid);
  }
  __syncthreads();
#pragma unroll
  for (int qq = 0; qq < PP; ++qq) {
    const int p = tid + qq * kThreads;
    if (p < ROWS * NP) {
      const int row = ROWS == 1 ? 0 : p / NP, k = ROWS == 1 ? p : p % NP;
      const Cx<CT> A = buf[pc(row * H + k)];
      const Cx<CT> B = buf[pc(row * H + ((H - k) & (H - 1)))];
      const CT xk = A.x * (k == 0 ? is0 : is1);
      const CT xnk = k > 0 ? A.y * is1 : (CT)0;
      const CT xp = (k == 0 ? A.y : B.x) * is1;
      const CT xnp = (k == 0 ? A.y : B.y) * is1;
      pre_pair<CT, H>({xk, -xnk}, {xp, -xnp}, k, tw, buf, row * H);
    }
  }
  __syncthreads();
  fft_rows<CT, H, ROWS, false>(buf, tw.fft, tid);
  constexpr int BATCH = NCH < 8 ? NCH : 8;
  static_assert(NCH % BATCH == 0, "output batches");
  if constexpr (OUT == 2) {
    const TO beta = (TO)st.sc[SC_BETA];
    const bool first = iter == 0;
#pragma unroll
    for (int b = 0; b < NCH; ++b) {
      const int e0 = (tid + b * kThreads) * W;
      const int row = e0 / N, c = e0 % N;
      if constexpr (!PRE) {
        if (!first) pv[b] = ld_nt<V>(q + (row0 + row) * ld + c);
        if (dupd) add_dir(b, pv[b]);
      }
      TO zo[W];
      if constexpr (W >= 4) {
        inv_chunk<CT, H, W, TO>(buf, row, c, inv_h, zo);
      } else {
#pragma unroll
        for (int t = 0; t < W; ++t) zo[t] = (TO)inv_value<CT, N>(v, row, c + t, inv_h);
      }
      V o;
#pragma unroll
      for (int t = 0; t < W; ++t) o[t] = first ? zo[t] : zo[t] + beta * pv[b][t];
      // a plain store: the operator reads p next, in part from the
      // last-level cache (measured 2% faster than a streaming store)
      *reinterpret_cast<V*>(z + (row0 + row) * ld + c) = o;
    }
    return;
  }
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i0 = 0; i0 < NCH; i0 += BATCH) {
    V rv[BATCH], qv[FLEX ? BATCH : 1];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      const int e0 = (tid + (i0 + b) * kThreads) * W;
      const int64_t o = (row0 + e0 / N) * ld + e0 % N;
      rv[b] = ld_nt<V>(r + o);
      if constexpr (FLEX) qv[b] = ld_nt<V>(q + o);
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      const int e0 = (tid + (i0 + b) * kThreads) * W;
      const int row = e0 / N, c = e0 % N;
      V zv;
      TO zo[W];
      if constexpr (W >= 4) {
        inv_chunk<CT, H, W, TO>(buf, row, c, inv_h, zo);
      } else {
#pragma unroll
        for (int t = 0; t < W; ++t) zo[t] = (TO)inv_value<CT, N>(v, row, c + t, inv_h);
      }
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const TO zt = zo[t];
        zv[t] = zt;
        const double zd = (double)zt;
        acc[0] += zd * (double)rv[b][t];
        if constexpr (FLEX) acc[1] += zd * (double)qv[b][t];
        acc[2] += zd;
      }
      st_nt<V>(z + (row0 + row) * ld + c, zv);
    }
  }
  const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
  write_partials<3>(st, slots, acc, (int)blockIdx.x);
}

// The n per-block partials of z.r, z.q, sum z folded into partial 0 (one
// block, fixed order), so that their consumers reduce a single value.
constexpr int kFoldThreads = 1024;
__global__ __launch_bounds__(kFoldThreads) void fct_fold_partials_kernel(DevState st, int n) {
  if (st.fl[FL_DONE]) return;
  const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double v = reduce_slot<kFoldThreads>(st, slots[i], n);
    if (threadIdx.x == 0) part_row(st, slots[i])[0] = v;
  }
}

// ---- transpose (square tiles through LDS) -------------------------------
// 16-byte loads along the input rows and 16-byte stores along the output
// rows; every load of a thread is issued before its first LDS write.  Tiles
// are 64 x 64 for 4- and 8-byte elements, 128 x 128 for 16-bit ones (32 KB
// of LDS either way).
template <class T>
constexpr int transpose_tile() {
  return sizeof(T) == 2 ? 128 : 64;
}

template <class T>
__device__ __forceinline__ void transpose_tile(const T* __restrict__ in, int64_t ldin,
                                               T* __restrict__ out, int64_t ldout) {
  using V = typename Vec16<T>::type;
  constexpr int TL = transpose_tile<T>();
  constexpr int W = Vec16<T>::W;
  constexpr int CPR = TL / W;            // chunks per tile row
  constexpr int RPP = kThreads / CPR;    // tile rows per pass
  constexpr int NPASS = TL / RPP;
  // row pitch TL + 2 elements: 16-bit tiles keep the column reads of a wave
  // on distinct 4-byte banks
  constexpr int PITCH = TL + (sizeof(T) == 2 ? 2 : 1);
  __shared__ T tile[TL][PITCH];
  const int64_t r0 = (int64_t)blockIdx.y * TL, c0 = (int64_t)blockIdx.x * TL;
  const int cq = threadIdx.x % CPR, rr = threadIdx.x / CPR;
  V d[NPASS];
#pragma unroll
  for (int i = 0; i < NPASS; ++i)
    d[i] = ld_nt<V>(in + (r0 + rr + i * RPP) * ldin + c0 + cq * W);
#pragma unroll
  for (int i = 0; i < NPASS; ++i)
#pragma unroll
    for (int t = 0; t < W; ++t) tile[rr + i * RPP][cq * W + t] = d[i][t];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NPASS; ++i) {
    const int jrow = rr + i * RPP;   // output row = input column c0 + jrow
    V o;
#pragma unroll
    for (int t = 0; t < W; ++t) o[t] = tile[cq * W + t][jrow];
    // a plain store: the next pass reads the transposed array, in part from
    // the last-level cache
    *reinterpret_cast<V*>(out + (c0 + jrow) * ldout + r0 + cq * W) = o;
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void transpose_kernel(const T* __restrict__ in, int64_t ldin,
                                                            T* __restrict__ out, int64_t ldout,
                                                            const int32_t* done) {
  if (*done) return;
  transpose_tile<T>(in, ldin, out, ldout);
}

// The transpose back after the column pass with the rho step (rho_body,
// 256 threads) in its first block: one launch and one dependent gap
// less per iteration.  A convergence found there makes the blocks that
// start later skip their tiles, which the last pass then does not read.
template <class T>
__global__ __launch_bounds__(kThreads) void transpose_rho_kernel(
    const T* __restrict__ in, int64_t ldin, T* __restrict__ out, int64_t ldout, DevState st,
    int n, int iter, int f16, int nparts_rr) {
  if (st.fl[FL_DONE]) return;
  if (blockIdx.x == 0 && blockIdx.y == 0) rho_body<kThreads>(st, n, iter, f16, nparts_rr);
  transpose_tile<T>(in, ldin, out, ldout);
}

template <class T>
static void launch_transpose(const T* in, int64_t rows, int64_t cols, T* out,
                             const int32_t* done, hipStream_t s) {
  constexpr int TL = transpose_tile<T>();
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)(cols / TL), (unsigned)(rows / TL)),
                     dim3(kThreads), 0, s, in, cols, out, rows, done);
}

template <class T>
void launch_transpose_any(const T* in, int64_t rows, int64_t cols, T* out, const int32_t* done,
                          hipStream_t s) {
  launch_transpose<T>(in, rows, cols, out, done, s);
}

template <class T>
void launch_transpose_rho(const T* in, int64_t rows, int64_t cols, T* out, DevState st, int n,
                          int iter, int f16, int nparts_rr, hipStream_t s) {
  constexpr int TL = transpose_tile<T>();
  hipLaunchKernelGGL(transpose_rho_kernel<T>, dim3((unsigned)(cols / TL), (unsigned)(rows / TL)),
                     dim3(kThreads), 0, s, in, cols, out, rows, st, n, iter, f16, nparts_rr);
}
template void launch_transpose_rho<double>(const double*, int64_t, int64_t, double*, DevState,
                                           int, int, int, int, hipStream_t);
template void launch_transpose_rho<float>(const float*, int64_t, int64_t, float*, DevState, int,
                                          int, int, int, hipStream_t);
template void launch_transpose_rho<_Float16>(const _Float16*, int64_t, int64_t, _Float16*,
                                             DevState, int, int, int, int, hipStream_t);
template void launch_transpose_rho<__bf16>(const __bf16*, int64_t, int64_t, __bf16*, DevState,
                                           int, int, int, int, hipStream_t);
template void launch_transpose_any<double>(const double*, int64_t, int64_t, double*,
                                           const int32_t*, hipStream_t);
template void launch_transpose_any<float>(const float*, int64_t, int64_t, float*, const int32_t*,
                                          hipStream_t);
template void launch_transpose_any<_Float16>(const _Float16*, int64_t, int64_t, _Float16*,
                                             const int32_t*, hipStream_t);
template void launch_transpose_any<__bf16>(const __bf16*, int64_t, int64_t, __bf16*,
                                           const int32_t*, hipStream_t);


void launch_fct_fold_partials(DevState st, int n, hipStream_t s) {
  hipLaunchKernelGGL(fct_fold_partials_kernel, dim3(1), dim3(kFoldThreads), 0, s, st, n);
}

void launch_cg_alpha(DevState st, int nparts_pq, int iter, int f16, double npix, hipStream_t s) {
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(1024), 0, s, st, nparts_pq, iter, f16, npix);
}

// ---- tables -----------------------------------------------------------------
// Thread j: stage-twiddle entry j (j < h - 1), post/pre twiddles j (j <= h),
// FP64 eigenvalue j (j < n), pair record j (j <= h/2), all from FP64.
template <class CT>
__global__ __launch_bounds__(kThreads) void fct_tables_kernel(int64_t n, Cx<CT>* tw, double* eig) {
  const int64_t h = n / 2;
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double s, c;
  if (j < h) {
    // stage with span ns and radix R holds entries ns - 1 .. ns R - 2
    int64_t ns = 1, rem = h, R = 1, num = 0;
    while (rem > 1) {
      R = rem >= 16 ? 16 : rem;
      if (j < ns * R - 1) {
        const int64_t rel = j - (ns - 1);
        num = (rel / ns + 1) * (rel % ns);   // r k
        break;
      }
      ns *= R;
      rem /= R;
    }
    if (j < h - 1) {
      sincospi(2.0 * (double)num / (double)(ns * R), &s, &c);
      tw[j] = {(CT)c, (CT)(-s)};
    } else {
      tw[j] = {(CT)0, (CT)0};
    }
  }
  if (j <= h) {
    sincospi(2.0 * (double)j / (double)n, &s, &c);
    tw[h + j] = {(CT)c, (CT)(-s)};
    sincospi(0.5 * (double)j / (double)n, &s, &c);
    tw[2 * h + 1 + j] = {(CT)c, (CT)(-s)};
  }
  if (j < n) {
    const double sv = sinpi(0.5 * (double)j / (double)n);
    eig[j] = 4.0 * sv * sv;
  }
  if (j <= h / 2)
    pair_tw_fill(reinterpret_cast<PairTw<CT>*>(reinterpret_cast<CT*>(tw) + pair_table_offset(h)) + j,
                 j, h, 2.0 * (double)n);
}

size_t fct_table_bytes(int64_t n, int elem) {
  const int64_t h = n / 2;
  return (size_t)pair_table_offset(h) * (size_t)elem +
         (size_t)(h / 2 + 1) * (elem == 8 ? sizeof(PairTw<double>) : sizeof(PairTw<float>));
}

void launch_fct_tables(int elem, int64_t n, void* tw, double* eig, hipStream_t s, bool general) {
  if (general) {
    launch_fctg_tables(elem, n, tw, eig, s);
    return;
  }
  const int nb = (int)((n + kThreads - 1) / kThreads);
  if (elem == 8)
    hipLaunchKernelGGL(fct_tables_kernel<double>, dim3(nb), dim3(kThreads), 0, s, n,
                       static_cast<Cx<double>*>(tw), eig);
  else
    hipLaunchKernelGGL(fct_tables_kernel<float>, dim3(nb), dim3(kThreads), 0, s, n,
                       static_cast<Cx<float>*>(tw), eig);
}

bool fct_supported(int64_t n) {
  return n >= 128 && n <= 16384 && (n & (n - 1)) == 0;
}

// ---- one application -----------------------------------------------------
template <class F>
static void with_h(int64_t h, F&& f) {
  switch (h) {
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    case 2048: f(std::integral_constant<int, 2048>{}); break;
    case 4096: f(std::integral_constant<int, 4096>{}); break;
    case 8192: f(std::integral_constant<int, 8192>{}); break;
    default: break;
  }
}

// CT: transform arithmetic; T: vector type (r, z, q); ST: storage of the
// two N x M intermediates (the plan's operand type: 16-bit for mixed plans,
// with the FP16 input scale of the prologue)
template <class CT, class T, class ST>
static int fast_impl(const PrecondArgs& a, hipStream_t s) {
  const int64_t N = a.N, M = a.M;
  const T* r = static_cast<const T*>(a.r);
  T* z = static_cast<T*>(a.z);
  const T* q = static_cast<const T*>(a.q);
  ST* T1 = static_cast<ST*>(a.T1);
  ST* T2 = static_cast<ST*>(a.T2);
  const int32_t* done = a.st.fl + FL_DONE;
  const int f16 = std::is_same<ST, _Float16>::value ? 1 : 0;
  LaunchLog* L = a.log;
  log_start(L, s);
  // fused head: pass 1 ran with the CG update and set the input scale; the
  // convergence test moves into the rho step
  if (!a.fused_head) {
    launch_fold_prologue(a.st, a.nparts_rr, a.check_conv, f16, N * M, s);
    log_mark(L, IRLSU_LK_PROLOGUE, s);
    with_h(M / 2, [&](auto hc) {
      constexpr int H = decltype(hc)::value;
      hipLaunchKernelGGL((fct_rows_fwd_kernel<CT, T, ST, H>),
                         dim3((unsigned)(N / rows_per_block<H>())), dim3(kThreads), 0, s, r, M,
                         T1, a.twM, done, f16 ? a.st.sc + SC_SCALE : nullptr);
    });
    log_mark(L, IRLSU_LK_ROWS_DCT2, s);
  }
  launch_transpose<ST>(T1, N, M, T2, done, s);
  log_mark(L, IRLSU_LK_TRANSPOSE, s);
  int ncols = 0;
  with_h(N / 2, [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    ncols = (int)(M / rows_per_block<H>());
    if (a.spectral)
      hipLaunchKernelGGL((fct_cols_kernel<CT, ST, H, true>), dim3((unsigned)ncols),
                         dim3(kThreads), 0, s, T2, N, a.twN,
                         static_cast<const double*>(a.eigM), a.st);
    else
      hipLaunchKernelGGL((fct_cols_kernel<CT, ST, H, false>), dim3((unsigned)ncols),
                         dim3(kThreads), 0, s, T2, N, a.twN,
                         static_cast<const double*>(a.eigM), a.st);
  });
  log_mark(L, IRLSU_LK_COLS, s);
  if (a.spectral)
    launch_transpose_rho<ST>(T2, M, N, T1, a.st, ncols, a.iter, f16,
                             a.fused_head && a.check_conv ? a.nparts_rr : 0, s);
  else
    launch_transpose<ST>(T2, M, N, T1, done, s);
  log_mark(L, IRLSU_LK_TRANSPOSE, s);
  int nb = 0;
  with_h(M / 2, [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    nb = (int)(N / rows_per_block<H>());
    if (a.spectral)
      hipLaunchKernelGGL((fct_rows_inv_kernel<CT, ST, T, H, 2>), dim3((unsigned)nb),
                         dim3(kThreads), 0, s, T1, M, static_cast<T*>(a.p_out), r,
                         static_cast<const T*>(a.p_in), static_cast<T*>(a.d), a.twM, a.st,
                         f16, a.iter);
    else if (q)
      hipLaunchKernelGGL((fct_rows_inv_kernel<CT, ST, T, H, 1>), dim3((unsigned)nb),
                         dim3(kThreads), 0, s, T1, M, z, r, q, nullptr, a.twM, a.st, f16, 0);
    else
      hipLaunchKernelGGL((fct_rows_inv_kernel<CT, ST, T, H, 0>), dim3((unsigned)nb),
                         dim3(kThreads), 0, s, T1, M, z, r, q, nullptr, a.twM, a.st, f16, 0);
  });
  log_mark(L, IRLSU_LK_ROWS_DCT3, s);
  if (!a.spectral) {
    hipLaunchKernelGGL(fct_fold_partials_kernel, dim3(1), dim3(kFoldThreads), 0, s, a.st, nb);
    log_mark(L, IRLSU_LK_PARTIALS, s);
  }
  return 1;
}

int fct_row_blocks(int64_t N, int64_t M) {
  if (!fct_supported(N) || !fct_supported(M)) return fctg_row_blocks(N, M);
  int nb = 0;
  with_h(M / 2, [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    nb = (int)(N / rows_per_block<H>());
  });
  return nb;
}

template <class CT, class T, class ST>
static int cg_update_impl(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter,
                          int nparts_out, hipStream_t s) {
  const int64_t N = a.N, M = a.M;
  const int f16 = std::is_same<ST, _Float16>::value ? 1 : 0;
  LaunchLog* L = a.log;
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(1024), 0, s, a.st, nparts_pq, iter, f16,
                     (double)(N * M));
  log_mark(L, IRLSU_LK_ALPHA, s);
  int nb = 0;
  with_h(M / 2, [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    nb = (int)(N / rows_per_block<H>());
    hipLaunchKernelGGL((fct_rows_fwd_cg_kernel<CT, T, ST, H>), dim3((unsigned)nb),
                       dim3(kThreads), 0, s, r, q, M, static_cast<ST*>(a.T1), a.twM, a.st, iter,
                       f16, nparts_out);
  });
  log_mark(L, IRLSU_LK_UPDATE_DCT2, s);
  return nb;
}

template <class T>
int launch_cg_update_fast(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter,
                          int nparts_out, hipStream_t s) {
  if (!fct_supported(a.N) || !fct_supported(a.M))
    return launch_cg_update_fastg<T>(a, r, q, nparts_pq, iter, nparts_out, s);
  if constexpr (std::is_same<T, double>::value) {
    return cg_update_impl<double, double, double>(a, r, q, nparts_pq, iter, nparts_out, s);
  } else {
    switch (a.kind) {
      case OK_F32:
        return cg_update_impl<float, float, float>(a, r, q, nparts_pq, iter, nparts_out, s);
      case OK_BF16:
        return cg_update_impl<float, float, __bf16>(a, r, q, nparts_pq, iter, nparts_out, s);
      case OK_F16:
        return cg_update_impl<float, float, _Float16>(a, r, q, nparts_pq, iter, nparts_out, s);
    }
    return 0;
  }
}
template int launch_cg_update_fast<float>(const PrecondArgs&, float*, const float*, int, int, int,
                                          hipStream_t);
template int launch_cg_update_fast<double>(const PrecondArgs&, double*, const double*, int, int,
                                           int, hipStream_t);

int launch_precond_fast(const PrecondArgs& a, hipStream_t s) {
  if (!fct_supported(a.N) || !fct_supported(a.M)) return launch_precond_fastg(a, s);
  switch (a.kind) {
    case OK_F64: return fast_impl<double, double, double>(a, s);
    case OK_F32: return fast_impl<float, float, float>(a, s);
    case OK_BF16: return fast_impl<float, float, __bf16>(a, s);
    case OK_F16: return fast_impl<float, float, _Float16>(a, s);
  }
  return 0;
}

}  // namespace irlsu
