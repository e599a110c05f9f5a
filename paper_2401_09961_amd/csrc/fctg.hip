// Fast form of the preconditioner (Section 3.3, Appendix B) for sides n = 2h
// that are not powers of two but whose half-length h has no prime factor
// above 5 (4000 = 2 x 2000 = 2 x 2^4 5^3, 6000, 16000, ...), n a multiple of
// 8 and h <= 8192.  The steps are those of the power-of-two passes of
// fct.hip -- even samples up and odd samples down, an h-point complex FFT,
// the twiddle post-processing to the orthonormal DCT-II coefficients, and
// the same backwards for the DCT-III -- with the FFT run as a sequence of
// Stockham stages of radix 16, 8, 4, 2, 5 and 3 whose plan (the radix list)
// is a launch argument, and every size a run-time value.
//
// Rows of a pass: floor(4096 / h) rows per block of 256 threads when
// h <= 4096, else one row per block of 512 threads (at most 4096 or 8192
// complex points of LDS).  Stage twiddles come from one table
// of the h-th roots of unity: the twiddle of point r of butterfly j in the
// stage of span NS and radix R is root[r (j mod NS) h / (NS R)].
//
// The intermediates T1, T2 are the plan's Np x Mp and Mp x Np buffers (both
// sides padded to multiples of 128): the row passes write the first N rows
// and M columns of T1, the transposes move the whole padded arrays and the
// column pass reads only the first M rows of T2, so the padding never meets
// the arithmetic.  The vectors keep the plan's row stride Mp.
#include "fft.hpp"
#include "kernels.hpp"

namespace irlsu {

namespace {

constexpr int kGMaxH = 8192;
constexpr int kGPts = 4096;
constexpr int kGMaxStages = 16;

struct GPlan {
  int h;
  int nst;
  int radix[kGMaxStages];
  // per stage, ceil(2^32 / d) for d = h / R (butterflies per row) and for
  // d = ns (the span): x / d = umulhi(x, m) exactly while x d < 2^32, which
  // holds here (x, d <= 8192); d = 1 is never divided by
  unsigned mag_bpr[kGMaxStages];
  unsigned mag_ns[kGMaxStages];
  // the same for the pairs per row (h/2 + 1) and the 16-byte chunks per row
  // (2h / W for W = 2, 4, 8 elements)
  unsigned mag_np;
  unsigned mag_c[3];
};

unsigned div_magic(int64_t d) {
  return d <= 1 ? 0u : (unsigned)((((uint64_t)1 << 32) + (uint64_t)d - 1) / (uint64_t)d);
}

// radices of an h-point FFT, first stage to last (false if h has a prime
// factor above 5)
bool make_plan(int64_t h, GPlan* p) {
  if (h < 4 || h > kGMaxH) return false;
  p->h = (int)h;
  p->nst = 0;
  int64_t rem = h;
  int64_t two = 1;
  while (rem % 2 == 0) {
    rem /= 2;
    two *= 2;
  }
  while (two > 1) {
    const int r = two >= 16 ? 16 : (int)two;
    p->radix[p->nst++] = r;
    two /= r;
  }
  for (int f : {5, 3}) {
    while (rem % f == 0) {
      rem /= f;
      if (p->nst == kGMaxStages) return false;
      p->radix[p->nst++] = f;
    }
  }
  p->mag_np = div_magic(h / 2 + 1);
  p->mag_c[0] = div_magic(h);
  p->mag_c[1] = div_magic(h / 2);
  p->mag_c[2] = div_magic(h / 4);
  int64_t ns = 1;
  for (int i = 0; i < p->nst; ++i) {
    p->mag_bpr[i] = div_magic(h / p->radix[i]);
    p->mag_ns[i] = div_magic(ns);
    ns *= p->radix[i];
  }
  return rem == 1;
}

// Threads per block: 256, or 512 for rows longer than 4096 points, whose
// 64 KiB of LDS (FP32) leave room for only two blocks per CU -- twice the
// waves to hide the latencies of the stages.
template <int CAP>
constexpr int g_threads() {
  return CAP > kGPts ? 512 : 256;
}

// blocks per CU that the LDS of one block leaves room for, as the register
// budget the kernels are compiled to (waves per SIMD: blocks x threads / 256)
template <class CT, int CAP>
constexpr int g_min_blocks() {
  return CAP * (int)sizeof(Cx<CT>) <= 32768 ? 4 : CAP * (int)sizeof(Cx<CT>) <= 65536 ? 2 : 1;
}

// x / d for a uniform divisor d with m = ceil(2^32 / d) (GPlan: exact for the
// index ranges that occur, x d < 2^32)
__device__ __forceinline__ int udiv(int x, int d, unsigned m) {
  return d == 1 ? x : (int)__umulhi((unsigned)x, m);
}
template <int W>
__device__ __forceinline__ unsigned chunk_magic(const GPlan& pl) {
  return pl.mag_c[W == 2 ? 0 : W == 4 ? 1 : 2];
}

__host__ __device__ inline int rows_per_block_g(int64_t h) {
  return h >= kGPts ? 1 : (int)(kGPts / h);
}

template <class CT>
struct GTw {
  const Cx<CT>* root;   // e^{-2 pi i m / h}, m < h
  const Cx<CT>* tn;     // e^{-2 pi i k / n}, k = 0..h
  const Cx<CT>* tq;     // e^{-i pi k / (2n)}, k = 0..h
  const PairTw<CT>* pair;  // the column pass's pair records, k = 0..h/2
};
template <class CT>
__device__ __forceinline__ GTw<CT> gtw_of(const void* p, int h) {
  const Cx<CT>* t = static_cast<const Cx<CT>*>(p);
  return {t, t + h, t + 2 * h + 1,
          reinterpret_cast<const PairTw<CT>*>(static_cast<const CT*>(p) + pair_table_offset(h))};
}

template <class CT, int R>
__device__ __forceinline__ void gdft(Cx<CT> (&a)[R]) {
  if constexpr (R == 3) {
    dft3(a[0], a[1], a[2]);
  } else if constexpr (R == 5) {
    dft5(a);
  } else {
    dft<CT, R>(a);
  }
}

// A copy of v the compiler cannot see through: index arithmetic derived from
// it after an FFT is not merged with the same arithmetic from before (which
// would hold those values in registers across all the stages).
__device__ __forceinline__ int opaque(int v) {
  int r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

// Twiddles of a butterfly, w[r] = root[r m] for r = 1..R-1 (r m < h): the
// powers 1, 2, 4 and 8 from the table (g_tw_load), the others as products
// of two of them (g_tw_expand, at most three roundings), which keeps a
// radix-16 butterfly at four table loads.
template <int R>
constexpr int g_tw_loads() {
  return R == 2 ? 1 : R <= 4 ? 2 : R <= 8 ? 3 : 4;
}
template <class CT, int R>
__device__ __forceinline__ void g_tw_load(const Cx<CT>* __restrict__ root, int m,
                                          Cx<CT> (&t)[g_tw_loads<R>()]) {
  t[0] = root[m];
  if constexpr (R > 2) t[1] = root[2 * m];
  if constexpr (R > 4) t[2] = root[4 * m];
  if constexpr (R > 8) t[3] = root[8 * m];
}
template <class CT, int R>
__device__ __forceinline__ void g_tw_expand(const Cx<CT> (&t)[g_tw_loads<R>()], Cx<CT> (&w)[R]) {
  w[1] = t[0];
  if constexpr (R > 2) w[2] = t[1];
  if constexpr (R > 3) w[3] = cmul(w[1], w[2]);
  if constexpr (R > 4) w[4] = t[2];
  if constexpr (R > 5) {
#pragma unroll
    for (int r = 5; r < 8; ++r) w[r] = cmul(w[4], w[r - 4]);
  }
  if constexpr (R > 8) {
    w[8] = t[3];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
  }
}

// One stage (span ns, radix R) over the block's rows, in place: butterfly j
// of a row reads points j + r h/R, multiplies point r by
// root[r (j mod ns) h / (ns R)], and writes its R-point DFT to
// (j - j mod ns) R + j mod ns + r ns.  A thread holds its butterflies in
// registers across the barrier; CAP bounds rows x h, hence their count.
// Straight-line loads: a butterfly index past the block's last one reads
// butterfly 0's points and twiddles (in range) and skips only its writes, so
// all of a thread's table and LDS loads are in flight before the first
// product instead of one butterfly's at a time.
template <class CT, int R, int CAP>
__device__ __forceinline__ void g_stage(Cx<CT>* buf, int h, int ns, int rows,
                                        const Cx<CT>* __restrict__ root, unsigned mag_bpr,
                                        unsigned mag_ns, int tid0) {
  const int tid = opaque(tid0);
  constexpr int NT = g_threads<CAP>();
  constexpr int NBM = (CAP / R + NT - 1) / NT;
  constexpr int NL = g_tw_loads<R>();
  // unsigned: the divisions by the uniform bpr and ns then need no sign fix
  const unsigned bpr = (unsigned)h / R, total = (unsigned)rows * bpr;
  const unsigned step = (unsigned)h / ((unsigned)ns * R), uns = (unsigned)ns;
  Cx<CT> a[NBM][R];
  Cx<CT> t[NBM][NL];
  int src[NBM], dst[NBM];
  bool act[NBM];
#pragma unroll
  for (int b = 0; b < NBM; ++b) {
    const unsigned bu = (unsigned)tid + (unsigned)b * NT;
    act[b] = bu < total;
    const unsigned bi = act[b] ? bu : 0u;
    const unsigned row = bpr == 1 ? bi : __umulhi(bi, mag_bpr);
    const unsigned j = bi - row * bpr;
    const unsigned k = uns == 1 ? 0u : j - __umulhi(j, mag_ns) * uns;
    src[b] = (int)(row * (unsigned)h + j);
    dst[b] = (int)(row * (unsigned)h + (j - k) * R + k);
    if (ns > 1) g_tw_load<CT, R>(root, (int)(k * step), t[b]);
  }
#pragma unroll
  for (int b = 0; b < NBM; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) a[b][r] = buf[src[b] + r * (int)bpr];
  }
#pragma unroll
  for (int b = 0; b < NBM; ++b) {
    if (ns > 1) {
      Cx<CT> w[R];
      g_tw_expand<CT, R>(t[b], w);
#pragma unroll
      for (int r = 1; r < R; ++r) a[b][r] = cmul(a[b][r], w[r]);
    }
    gdft<CT, R>(a[b]);
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NBM; ++b) {
    if (act[b]) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[b] + r * ns] = a[b][r];
    }
  }
  __syncthreads();
}

template <class CT, int CAP>
__device__ __forceinline__ void g_fft(Cx<CT>* buf, const GPlan& pl, int rows,
                                      const Cx<CT>* __restrict__ root, int tid) {
  int ns = 1;
#pragma nounroll
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.radix[s];
    const unsigned mb = pl.mag_bpr[s], mn = pl.mag_ns[s];
    switch (R) {
      case 16: g_stage<CT, 16, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
      case 8: g_stage<CT, 8, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
      case 4: g_stage<CT, 4, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
      case 2: g_stage<CT, 2, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
      case 5: g_stage<CT, 5, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
      default: g_stage<CT, 3, CAP>(buf, pl.h, ns, rows, root, mb, mn, tid); break;
    }
    ns *= R;
  }
}

// position of row element e in the even-up / odd-down sequence (length n)
__device__ __forceinline__ int gperm(int e, int n) { return (e & 1) ? n - 1 - (e >> 1) : (e >> 1); }

// Pair steps of one row held in LDS (post_core and pre_core), the twiddles
// from the side's tables, as post_pair and pre_pair in fct.hip.
template <class CT>
__device__ __forceinline__ void g_post_pair(const Cx<CT>* row, int h, int k, const GTw<CT>& tw,
                                            Cx<CT>& ck, Cx<CT>& cp) {
  post_core(row[k], row[k == 0 ? 0 : h - k], tw.tq[k], tw.tq[h - k], tw.tn[k], ck, cp);
}

template <class CT>
__device__ __forceinline__ void g_pre_pair(Cx<CT> ck, Cx<CT> cp, int h, int k, const GTw<CT>& tw,
                                           Cx<CT>* row) {
  Cx<CT> sk, sp;
  pre_core(ck, cp, tw.tq[k], tw.tq[h - k], tw.tn[k], sk, sp);
  row[k] = sk;
  if (k != h - k && k > 0) row[h - k] = sp;
}

// Streams the block's rows (n elements each, 16-byte chunks) through f(row,
// column, chunk), eight chunks per thread in flight at a time.
template <class TI, int NT, class F>
__device__ __forceinline__ void g_rows_in(const TI* __restrict__ in, int64_t ld, int64_t row0,
                                          int rows, int n, unsigned mcpr, int tid, F&& f) {
  using V = typename Vec16<TI>::type;
  constexpr int W = Vec16<TI>::W;
  const int cpr = n / W, total = rows * cpr;
  for (int base = 0; base < total; base += 8 * NT) {
    V d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int ci = base + tid + u * NT;
      if (ci < total) {
        const int row = udiv(ci, cpr, mcpr), c = (ci - row * cpr) * W;
        d[u] = ld_nt<V>(in + (row0 + row) * ld + c);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int ci = base + tid + u * NT;
      if (ci < total) {
        const int row = udiv(ci, cpr, mcpr), c = (ci - row * cpr) * W;
        f(row, c, d[u]);
      }
    }
  }
}

// LDS <- chunk of W elements at column c of a row, in the even-up /
// odd-down order, times scale (put_rows of fct.hip)
template <class CT, class V, int W>
__device__ __forceinline__ void g_put(Cx<CT>* buf, int h, int row, int c, const V& d, CT scale) {
  Cx<CT>* b = buf + row * h;
  if constexpr (W >= 4) {
#pragma unroll
    for (int s4 = 0; s4 < W / 4; ++s4) {
      b[c / 4 + s4] = {(CT)d[4 * s4] * scale, (CT)d[4 * s4 + 2] * scale};
      b[h - 1 - c / 4 - s4] = {(CT)d[4 * s4 + 3] * scale, (CT)d[4 * s4 + 1] * scale};
    }
  } else {
    CT* v = reinterpret_cast<CT*>(b);
#pragma unroll
    for (int t = 0; t < W; ++t) v[gperm(c + t, 2 * h)] = (CT)d[t] * scale;
  }
}

// LDS <- chunk for the inverse pre-processing (put_rows_inv of fct.hip):
// element e to slot e (real part) for e < h, to slot (n - e) mod h
// (imaginary part) for e >= h
template <class CT, class V, int W>
__device__ __forceinline__ void g_put_inv(Cx<CT>* buf, int h, int row, int c, const V& d) {
  CT* v = reinterpret_cast<CT*>(buf + row * h);
  const int n = 2 * h;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int e = c + t;
    const int slot = e < h ? e : (e == h ? 0 : n - e);
    v[2 * slot + (e < h ? 0 : 1)] = (CT)d[t];
  }
}

// W output elements at column c of a row after the inverse FFT (inv_chunk /
// inv_value of fct.hip)
template <class CT, int W, class OT>
__device__ __forceinline__ void g_inv_chunk(const Cx<CT>* buf, int h, int row, int c, CT inv_h,
                                            OT (&o)[W]) {
  const Cx<CT>* b = buf + row * h;
  if constexpr (W >= 4) {
#pragma unroll
    for (int s4 = 0; s4 < W / 4; ++s4) {
      const Cx<CT> A = b[c / 4 + s4];
      const Cx<CT> B = b[h - 1 - c / 4 - s4];
      o[4 * s4] = (OT)(A.x * inv_h);
      o[4 * s4 + 1] = (OT)(-B.y * inv_h);
      o[4 * s4 + 2] = (OT)(-A.y * inv_h);
      o[4 * s4 + 3] = (OT)(B.x * inv_h);
    }
  } else {
    const CT* v = reinterpret_cast<const CT*>(b);
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int m = gperm(c + t, 2 * h);
      const CT x = v[m];
      o[t] = (OT)(((m & 1) ? -x : x) * inv_h);
    }
  }
}

// DCT-II outputs of the block's rows from the FFT in LDS: X_k = s_k Re c_k,
// X_{n-k} = -s_k Im c_k (twice c from the post-processing, so s/2)
template <class CT, class TO, int NT>
__device__ __forceinline__ void g_store_dct2(const Cx<CT>* buf, int h, int rows, const GTw<CT>& tw,
                                             TO* __restrict__ out, int64_t ldo, int64_t row0,
                                             unsigned mnp, int tid) {
  const int n = 2 * h, np = h / 2 + 1;
  const CT s0 = (CT)(0.5 * sqrt(1.0 / n)), s1 = (CT)(0.5 * sqrt(2.0 / n));
  for (int p = tid; p < rows * np; p += NT) {
    const int row = udiv(p, np, mnp), k = p - row * np;
    Cx<CT> ck, cp;
    g_post_pair<CT>(buf + row * h, h, k, tw, ck, cp);
    TO* o = out + (row0 + row) * ldo;
    o[k] = (TO)(ck.x * (k == 0 ? s0 : s1));
    if (k > 0) o[n - k] = (TO)(-ck.y * s1);
    if (h - k != k) {
      o[h - k] = (TO)(cp.x * s1);
      if (k > 0) o[h + k] = (TO)(-cp.y * s1);
    }
  }
}

// ---- pass 1: DCT-II along rows ---------------------------------------------
template <class CT, class TI, class TO, int CAP>
__global__ __launch_bounds__(g_threads<CAP>(), (g_min_blocks<CT, CAP>())) void g_rows_fwd_kernel(
    const TI* __restrict__ in, int64_t ld, TO* __restrict__ out, int64_t ldo, int64_t nrows,
    GPlan pl, const void* twp, const int32_t* done, const double* scale_p) {
  constexpr int NT = g_threads<CAP>();
  if (*done) return;
  __shared__ Cx<CT> buf[CAP];
  const int h = pl.h, tid = threadIdx.x;
  const int rpb = rows_per_block_g(h);
  const int64_t row0 = (int64_t)blockIdx.x * rpb;
  const int rows = (int)(nrows - row0 < rpb ? nrows - row0 : rpb);
  const GTw<CT> tw = gtw_of<CT>(twp, h);
  const CT scale = scale_p ? (CT)*scale_p : (CT)1;
  using V = typename Vec16<TI>::type;
  constexpr int W = Vec16<TI>::W;
  g_rows_in<TI, NT>(in, ld, row0, rows, 2 * h, chunk_magic<W>(pl), tid,
                [&](int row, int c, const V& d) { g_put<CT, V, W>(buf, h, row, c, d, scale); });
  __syncthreads();
  g_fft<CT, CAP>(buf, pl, rows, tw.root, tid);
  g_store_dct2<CT, TO, NT>(buf, h, rows, tw, out, ldo, row0, pl.mag_np, opaque(tid));
}

// ---- CG update fused with pass 1 (fct_rows_fwd_cg_kernel) --------------------
template <class CT, class T, class TO, int CAP>
__global__ __launch_bounds__(g_threads<CAP>(), (g_min_blocks<CT, CAP>())) void g_rows_fwd_cg_kernel(
    T* __restrict__ r, const T* __restrict__ q, int64_t ld, TO* __restrict__ out, int64_t ldo,
    int64_t nrows, GPlan pl, const void* twp, DevState st, int iter, int f16, int nparts_out) {
  constexpr int NT = g_threads<CAP>();
  if (st.fl[FL_DONE]) return;
  __shared__ Cx<CT> buf[CAP];
  const int h = pl.h, n = 2 * h, tid = threadIdx.x;
  const int rpb = rows_per_block_g(h);
  const int64_t row0 = (int64_t)blockIdx.x * rpb;
  const int rows = (int)(nrows - row0 < rpb ? nrows - row0 : rpb);
  const GTw<CT> tw = gtw_of<CT>(twp, h);
  const T al = (T)st.sc[SC_ALPHA + (iter & 1)];
  const CT scale = f16 ? (CT)st.sc[SC_SCALE] : (CT)1;
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::W;
  double acc[2] = {0.0, 0.0};
  const int cpr = n / W, total = rows * cpr;
  for (int base = 0; base < total; base += 4 * NT) {
    V qv[4], rv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ci = base + tid + u * NT;
      if (ci < total) {
        const int row = udiv(ci, cpr, chunk_magic<W>(pl)), c = (ci - row * cpr) * W;
        const int64_t o = (row0 + row) * ld + c;
        qv[u] = ld_nt<V>(q + o);
        rv[u] = ld_nt<V>(r + o);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ci = base + tid + u * NT;
      if (ci < total) {
        const int row = udiv(ci, cpr, chunk_magic<W>(pl)), c = (ci - row * cpr) * W;
#pragma unroll
        for (int t = 0; t < W; ++t) {
          rv[u][t] = rv[u][t] - al * qv[u][t];
          acc[0] += (double)rv[u][t] * (double)rv[u][t];
          acc[1] += (double)rv[u][t];
        }
        st_nt<V>(r + (row0 + row) * ld + c, rv[u]);
        g_put<CT, V, W>(buf, h, row, c, rv[u], scale);
      }
    }
  }
  __syncthreads();
  g_fft<CT, CAP>(buf, pl, rows, tw.root, tid);
  g_store_dct2<CT, TO, NT>(buf, h, rows, tw, out, ldo, row0, pl.mag_np, opaque(tid));
  const int slots[2] = {PR_RR, PR_RSUM};
  write_partials<2, NT>(st, slots, acc, (int)blockIdx.x);
  if (threadIdx.x == 0) {
    for (int k = (int)blockIdx.x + (int)gridDim.x; k < nparts_out; k += (int)gridDim.x) {
      part_row(st, PR_RR)[k] = 0.0;
      part_row(st, PR_RSUM)[k] = 0.0;
    }
  }
}

// ---- pass 3: DCT-II, spectral division, DCT-III along the rows of the
// transposed intermediate (fct_cols_kernel) ---------------------------------
template <class CT, class ST, int CAP, bool RHO>
__global__ __launch_bounds__(g_threads<CAP>(), (g_min_blocks<CT, CAP>())) void g_cols_kernel(
    ST* __restrict__ io, int64_t ld, int64_t nrows, GPlan pl, const void* twp,
    const double* __restrict__ eig_l, DevState st) {
  constexpr int NT = g_threads<CAP>();
  if (st.fl[FL_DONE]) return;
  __shared__ Cx<CT> buf[CAP];
  const int h = pl.h, n = 2 * h, tid = threadIdx.x;
  const int rpb = rows_per_block_g(h);
  const int64_t row0 = (int64_t)blockIdx.x * rpb;
  const int rows = (int)(nrows - row0 < rpb ? nrows - row0 : rpb);
  const GTw<CT> tw = gtw_of<CT>(twp, h);
  using V = typename Vec16<ST>::type;
  constexpr int W = Vec16<ST>::W;
  g_rows_in<ST, NT>(io, ld, row0, rows, n, chunk_magic<W>(pl), tid,
                [&](int row, int c, const V& d) { g_put<CT, V, W>(buf, h, row, c, d, (CT)1); });
  __syncthreads();
  g_fft<CT, CAP>(buf, pl, rows, tw.root, tid);
  CT rho = (CT)0;
  const int np = h / 2 + 1;
  for (int p = opaque(tid); p < rows * np; p += NT) {
    const int row = udiv(p, np, pl.mag_np), k = p - row * np;
    const int64_t l = row0 + row;
    const CT mu = (CT)eig_l[l];
    const PairTw<CT> pt = tw.pair[k];
    Cx<CT>* slot_k = buf + row * h + k;
    Cx<CT>* slot_p = buf + row * h + (k == 0 ? 0 : h - k);
    Cx<CT> ck, cp;
    post_core(*slot_k, *slot_p, pt.q, pt.qp, pt.n, ck, cp);
    const CT dk = (l == 0 && k == 0) ? (CT)0 : recip(pt.e[0] + mu);
    const CT dnk = k > 0 ? recip(pt.e[1] + mu) : (CT)0;
    const CT dp = recip(pt.e[2] + mu), dnp = recip(pt.e[3] + mu);
    const CT xk = ck.x * dk;
    const CT xnk = k > 0 ? -ck.y * dnk : (CT)0;
    const CT xp = cp.x * dp;
    const CT xnp = -cp.y * dnp;
    Cx<CT> sk, sp;
    pre_core<CT>({xk, -xnk}, {xp, -xnp}, pt.q, pt.qp, pt.n, sk, sp);
    *slot_k = sk;
    if (k != h - k && k > 0) *slot_p = sp;
    if constexpr (RHO) {
      rho += (k == 0 ? (CT)0.5 : (CT)1) * ck.x * ck.x * dk;
      if (k > 0) rho += ck.y * ck.y * dnk;
      if (k < h / 2) rho += cp.x * cp.x * dp;
      if (k > 0 && k < h / 2) rho += cp.y * cp.y * dnp;
    }
  }
  __syncthreads();
  g_fft<CT, CAP>(buf, pl, rows, tw.root, tid);
  const CT inv_h = (CT)(0.25 / h);
  const int cpr = n / W;
  for (int ci = opaque(tid); ci < rows * cpr; ci += NT) {
    const int row = udiv(ci, cpr, chunk_magic<W>(pl)), c = (ci - row * cpr) * W;
    ST ot[W];
    g_inv_chunk<CT, W, ST>(buf, h, row, c, inv_h, ot);
    V o;
#pragma unroll
    for (int t = 0; t < W; ++t) o[t] = ot[t];
    *reinterpret_cast<V*>(io + (row0 + row) * ld + c) = o;
  }
  if constexpr (RHO) {
    double acc[1] = {(double)rho * (0.5 / (double)n)};
    const int slots[1] = {PR_ZR};
    write_partials<1, NT>(st, slots, acc, (int)blockIdx.x);
  }
}

// ---- pass 5: DCT-III along rows (fct_rows_inv_kernel) -------------------------
// OUT 0: z and the dots z.r, sum z; 1: also z.q; 2: the direction p = z +
// beta p_in into z (p_in passed as q, unread at iter 0), and with dacc
// non-null dacc += alpha_{iter-1} p_in -- alone if the rho step stopped the
// solve on convergence (FL_DPEND).
template <class CT, class SI, class TO, int CAP, int OUT>
__global__ __launch_bounds__(g_threads<CAP>(), (g_min_blocks<CT, CAP>())) void g_rows_inv_kernel(
    const SI* __restrict__ in, int64_t ldi, TO* __restrict__ z, int64_t ld,
    const TO* __restrict__ r, const TO* __restrict__ q, TO* __restrict__ dacc, int64_t nrows,
    int64_t nrows_pad, GPlan pl, const void* twp, DevState st, int use_scale, int iter) {
  constexpr int NT = g_threads<CAP>();
  const int h = pl.h, n = 2 * h, tid = threadIdx.x;
  const int rpb = rows_per_block_g(h);
  const int64_t row0 = (int64_t)blockIdx.x * rpb;
  const int rows = (int)(nrows - row0 < rpb ? nrows - row0 : rpb);
  using V = typename Vec16<TO>::type;
  constexpr int W = Vec16<TO>::W;
  const int cpr = n / W, total = rows * cpr;
  const bool dupd = OUT == 2 && dacc != nullptr && iter != 0;
  const TO al = dupd ? (TO)st.sc[SC_ALPHA + ((iter - 1) & 1)] : (TO)0;
  auto add_dir = [&](int ci) {
    const int row = udiv(ci, cpr, chunk_magic<W>(pl)), c = (ci - row * cpr) * W;
    const int64_t o = (row0 + row) * ld + c;
    const V pv = ld_nt<V>(q + o);
    V dv = ld_nt<V>(dacc + o);
#pragma unroll
    for (int t = 0; t < W; ++t) dv[t] = dv[t] + al * pv[t];
    st_nt<V>(dacc + o, dv);
  };
  if (st.fl[FL_DONE]) {
    if (dupd && st.fl[FL_DPEND]) {
      for (int ci = tid; ci < total; ci += NT) add_dir(ci);
    }
    return;
  }
  __shared__ Cx<CT> buf[CAP];
  const GTw<CT> tw = gtw_of<CT>(twp, h);
  const CT inv_h = (CT)(0.5 / h) / (use_scale ? (CT)st.sc[SC_SCALE] : (CT)1);
  const CT is0 = (CT)sqrt((double)n), is1 = (CT)sqrt(0.5 * n);
  using VI = typename Vec16<SI>::type;
  constexpr int WI = Vec16<SI>::W;
  g_rows_in<SI, NT>(in, ldi, row0, rows, n, chunk_magic<WI>(pl), tid,
                [&](int row, int c, const VI& d) { g_put_inv<CT, VI, WI>(buf, h, row, c, d); });
  __syncthreads();
  const int np = h / 2 + 1;
  for (int p = opaque(tid); p < rows * np; p += NT) {
    const int row = udiv(p, np, pl.mag_np), k = p - row * np;
    const Cx<CT>* b = buf + row * h;
    const Cx<CT> A = b[k];
    const Cx<CT> B = b[k == 0 ? 0 : h - k];
    const CT xk = A.x * (k == 0 ? is0 : is1);
    const CT xnk = k > 0 ? A.y * is1 : (CT)0;
    const CT xp = (k == 0 ? A.y : B.x) * is1;
    const CT xnp = (k == 0 ? A.y : B.y) * is1;
    g_pre_pair<CT>({xk, -xnk}, {xp, -xnp}, h, k, tw, buf + row * h);
  }
  __syncthreads();
  g_fft<CT, CAP>(buf, pl, rows, tw.root, tid);
  double acc[3] = {0.0, 0.0, 0.0};
  const TO beta = OUT == 2 ? (TO)st.sc[SC_BETA] : (TO)0;
  for (int ci = opaque(tid); ci < total; ci += NT) {
    const int row = udiv(ci, cpr, chunk_magic<W>(pl)), c = (ci - row * cpr) * W;
    const int64_t o = (row0 + row) * ld + c;
    TO zo[W];
    g_inv_chunk<CT, W, TO>(buf, h, row, c, inv_h, zo);
    V out;
    if constexpr (OUT == 2) {
      if (iter != 0) {
        // p_in once, for the new direction and for the iterate update
        const V pv = ld_nt<V>(q + o);
        if (dupd) {
          V dv = ld_nt<V>(dacc + o);
#pragma unroll
          for (int t = 0; t < W; ++t) dv[t] = dv[t] + al * pv[t];
          st_nt<V>(dacc + o, dv);
        }
#pragma unroll
        for (int t = 0; t < W; ++t) out[t] = zo[t] + beta * pv[t];
      } else {
#pragma unroll
        for (int t = 0; t < W; ++t) out[t] = zo[t];
      }
    } else {
      const V rv = ld_nt<V>(r + o);
      V qv;
      if constexpr (OUT == 1) qv = ld_nt<V>(q + o);
#pragma unroll
      for (int t = 0; t < W; ++t) {
        out[t] = zo[t];
        const double zd = (double)zo[t];
        acc[0] += zd * (double)rv[t];
        if constexpr (OUT == 1) acc[1] += zd * (double)qv[t];
        acc[2] += zd;
      }
    }
    if constexpr (OUT == 2)
      *reinterpret_cast<V*>(z + o) = out;   // read by the operator next (as in fct.hip)
    else
      st_nt<V>(z + o, out);
  }
  // zeros in the output's padding, as the product forms leave it: columns
  // [n, ld) of the block's rows, and the rows [nrows, nrows_pad) spread over
  // the blocks
  const int padc = (int)(ld - n);
  for (int i = opaque(tid); i < rows * padc; i += NT) {
    const int row = i / padc;
    z[(row0 + row) * ld + n + (i - row * padc)] = (TO)0;
  }
  for (int64_t pr = nrows + blockIdx.x; pr < nrows_pad; pr += gridDim.x)
    for (int64_t j = tid; j < ld; j += NT) z[pr * ld + j] = (TO)0;
  if constexpr (OUT != 2) {
    const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
    write_partials<3, NT>(st, slots, acc, (int)blockIdx.x);
  }
}

// ---- tables -------------------------------------------------------------------
// Layout of fct_tables_kernel (fct.hip) with the h roots of unity in place of
// the power-of-two stage twiddles: [0, h) e^{-2 pi i m/h}; [h, 2h]
// e^{-2 pi i k/n}; [2h+1, 3h+1] e^{-i pi k/(2n)}; the h/2 + 1 pair records
// (PairTw, eigenvalues unscaled: the output pass applies 1/(4h)); and the
// FP64 eigenvalues in eig.
template <class CT>
__global__ __launch_bounds__(kThreads) void g_tables_kernel(int64_t n, Cx<CT>* tw, double* eig) {
  const int64_t h = n / 2;
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double s, c;
  if (j < h) {
    sincospi(2.0 * (double)j / (double)h, &s, &c);
    tw[j] = {(CT)c, (CT)(-s)};
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
                 j, h, 1.0);
}

template <class F>
void with_cap(int64_t h, F&& f) {
  if (h > kGPts)
    f(std::integral_constant<int, kGMaxH>{});
  else
    f(std::integral_constant<int, kGPts>{});
}

int blocks_g(int64_t nrows, int64_t h) {
  const int rpb = rows_per_block_g(h);
  return (int)((nrows + rpb - 1) / rpb);
}

template <class CT, class T, class ST>
int fastg_impl(const PrecondArgs& a, hipStream_t s) {
  const int64_t N = a.N, M = a.M, Np = a.Np, Mp = a.Mp;
  GPlan pN, pM;
  if (!make_plan(N / 2, &pN) || !make_plan(M / 2, &pM)) return 0;
  const T* r = static_cast<const T*>(a.r);
  T* z = static_cast<T*>(a.z);
  const T* q = static_cast<const T*>(a.q);
  ST* T1 = static_cast<ST*>(a.T1);
  ST* T2 = static_cast<ST*>(a.T2);
  const int32_t* done = a.st.fl + FL_DONE;
  const int f16 = std::is_same<ST, _Float16>::value ? 1 : 0;
  LaunchLog* L = a.log;
  log_start(L, s);
  if (!a.fused_head) {
    launch_fold_prologue(a.st, a.nparts_rr, a.check_conv, f16, N * M, s);
    log_mark(L, IRLSU_LK_PROLOGUE, s);
    with_cap(M / 2, [&](auto cap) {
      constexpr int CAP = decltype(cap)::value;
      hipLaunchKernelGGL((g_rows_fwd_kernel<CT, T, ST, CAP>), dim3(blocks_g(N, M / 2)),
                         dim3(g_threads<CAP>()), 0, s, r, Mp, T1, Mp, N, pM, a.twM, done,
                         f16 ? a.st.sc + SC_SCALE : nullptr);
    });
    log_mark(L, IRLSU_LK_ROWS_DCT2, s);
  }
  launch_transpose_any<ST>(T1, Np, Mp, T2, done, s);
  log_mark(L, IRLSU_LK_TRANSPOSE, s);
  const int ncols = blocks_g(M, N / 2);
  with_cap(N / 2, [&](auto cap) {
    constexpr int CAP = decltype(cap)::value;
    if (a.spectral)
      hipLaunchKernelGGL((g_cols_kernel<CT, ST, CAP, true>), dim3(ncols),
                         dim3(g_threads<CAP>()), 0, s,
                         T2, Np, M, pN, a.twN, static_cast<const double*>(a.eigM), a.st);
    else
      hipLaunchKernelGGL((g_cols_kernel<CT, ST, CAP, false>), dim3(ncols),
                         dim3(g_threads<CAP>()), 0, s,
                         T2, Np, M, pN, a.twN, static_cast<const double*>(a.eigM), a.st);
  });
  log_mark(L, IRLSU_LK_COLS, s);
  if (a.spectral)
    launch_transpose_rho<ST>(T2, Mp, Np, T1, a.st, ncols, a.iter, f16,
                             a.fused_head && a.check_conv ? a.nparts_rr : 0, s);
  else
    launch_transpose_any<ST>(T2, Mp, Np, T1, done, s);
  log_mark(L, IRLSU_LK_TRANSPOSE, s);
  const int nb = blocks_g(N, M / 2);
  with_cap(M / 2, [&](auto cap) {
    constexpr int CAP = decltype(cap)::value;
    if (a.spectral)
      hipLaunchKernelGGL((g_rows_inv_kernel<CT, ST, T, CAP, 2>), dim3(nb),
                         dim3(g_threads<CAP>()), 0, s,
                         T1, Mp, static_cast<T*>(a.p_out), Mp, r, static_cast<const T*>(a.p_in),
                         static_cast<T*>(a.d), N, Np, pM, a.twM, a.st, f16, a.iter);
    else if (q)
      hipLaunchKernelGGL((g_rows_inv_kernel<CT, ST, T, CAP, 1>), dim3(nb),
                         dim3(g_threads<CAP>()), 0, s,
                         T1, Mp, z, Mp, r, q, nullptr, N, Np, pM, a.twM, a.st, f16, 0);
    else
      hipLaunchKernelGGL((g_rows_inv_kernel<CT, ST, T, CAP, 0>), dim3(nb),
                         dim3(g_threads<CAP>()), 0, s,
                         T1, Mp, z, Mp, r, q, nullptr, N, Np, pM, a.twM, a.st, f16, 0);
  });
  log_mark(L, IRLSU_LK_ROWS_DCT3, s);
  if (!a.spectral) {
    launch_fct_fold_partials(a.st, nb, s);
    log_mark(L, IRLSU_LK_PARTIALS, s);
  }
  return 1;
}

template <class CT, class T, class ST>
int cg_update_g(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter, int nparts_out,
                hipStream_t s) {
  const int64_t N = a.N, M = a.M, Mp = a.Mp;
  GPlan pM;
  if (!make_plan(M / 2, &pM)) return 0;
  const int f16 = std::is_same<ST, _Float16>::value ? 1 : 0;
  launch_cg_alpha(a.st, nparts_pq, iter, f16, (double)(N * M), s);
  log_mark(a.log, IRLSU_LK_ALPHA, s);
  const int nb = blocks_g(N, M / 2);
  with_cap(M / 2, [&](auto cap) {
    constexpr int CAP = decltype(cap)::value;
    hipLaunchKernelGGL((g_rows_fwd_cg_kernel<CT, T, ST, CAP>), dim3(nb),
                       dim3(g_threads<CAP>()), 0, s, r, q, Mp, static_cast<ST*>(a.T1), Mp, N,
                       pM, a.twM, a.st, iter, f16, nparts_out);
  });
  log_mark(a.log, IRLSU_LK_UPDATE_DCT2, s);
  return nb;
}

}  // namespace

bool fctg_supported(int64_t n) {
  GPlan p;
  return n % 8 == 0 && make_plan(n / 2, &p);
}

int fctg_row_blocks(int64_t N, int64_t M) { return blocks_g(N, M / 2); }

void launch_fctg_tables(int elem, int64_t n, void* tw, double* eig, hipStream_t s) {
  const int nb = (int)((n + kThreads - 1) / kThreads);
  if (elem == 8)
    hipLaunchKernelGGL(g_tables_kernel<double>, dim3(nb), dim3(kThreads), 0, s, n,
                       static_cast<Cx<double>*>(tw), eig);
  else
    hipLaunchKernelGGL(g_tables_kernel<float>, dim3(nb), dim3(kThreads), 0, s, n,
                       static_cast<Cx<float>*>(tw), eig);
}

int launch_precond_fastg(const PrecondArgs& a, hipStream_t s) {
  switch (a.kind) {
    case OK_F64: return fastg_impl<double, double, double>(a, s);
    case OK_F32: return fastg_impl<float, float, float>(a, s);
    case OK_BF16: return fastg_impl<float, float, __bf16>(a, s);
    case OK_F16: return fastg_impl<float, float, _Float16>(a, s);
  }
  return 0;
}

template <class T>
int launch_cg_update_fastg(const PrecondArgs& a, T* r, const T* q, int nparts_pq, int iter,
                           int nparts_out, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    return cg_update_g<double, double, double>(a, r, q, nparts_pq, iter, nparts_out, s);
  } else {
    switch (a.kind) {
      case OK_F32: return cg_update_g<float, float, float>(a, r, q, nparts_pq, iter, nparts_out, s);
      case OK_BF16:
        return cg_update_g<float, float, __bf16>(a, r, q, nparts_pq, iter, nparts_out, s);
      case OK_F16:
        return cg_update_g<float, float, _Float16>(a, r, q, nparts_pq, iter, nparts_out, s);
    }
    return 0;
  }
}
template int launch_cg_update_fastg<float>(const PrecondArgs&, float*, const float*, int, int,
                                           int, hipStream_t);
template int launch_cg_update_fastg<double>(const PrecondArgs&, double*, const double*, int, int,
                                            int, hipStream_t);

}  // namespace irlsu
