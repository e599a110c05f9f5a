// Preconditioner z = L^+ r of Section 3.3: with the eigendecompositions
// S^T S = P_N Lambda_N P_N^T and T T^T = P_M Lambda_M P_M^T (P the orthonormal
// DCT-II basis), z = P_N [ (P_N^T r P_M) ./ (lambda_k + mu_l) ] P_M^T, mode
// (0,0) set to zero (the pseudo-inverse choice of Appendix B).  The paper
// names the two dense products as the bottleneck; here they are four dense
// GEMMs on the MFMA units, every one in "NT" form (both operands contiguous
// along the contraction index), chaining transposed and direct stores:
//
//   G1  T1^T[l][i] = sum_j r[i][j]   P_M[j][l]      (A = r, B = P_M^T)
//   G2  T2^T[l][k] = sum_i T1^T[l][i] P_N[i][k] / (lambda_k + mu_l)
//   G3  T3[i][l]   = sum_k T2^T[l][k] P_N[i][k]     (B = P_N)
//   G4  z[i][j]    = sum_l T3[i][l]  P_M[j][l]      (B = P_M), epilogue
//                    partial sums z.r, z.q, sum z in FP64
//
// Operand precisions: FP64 (v_mfma_f64_16x16x4f64), FP32
// (v_mfma_f32_32x32x2f32), BF16 / FP16 (v_mfma_f32_32x32x16_{bf16,f16}) with
// FP32 accumulation; intermediates are stored in the operand type.
#include <type_traits>

#include "kernels.hpp"

namespace irlsu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class OT>
struct Mfma;

// Result layout of the 32 x 32 instructions: accumulator e of lane l holds
// row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32 (RS = 1: the four values
// of a group are consecutive rows).  The FP64 16 x 16 x 4 instruction holds
// row 4 e + l / 16, column l % 16 (RS = 4).
template <>
struct Mfma<__bf16> {
  static constexpr int TM = 32, KPL = 8, TK = 16, NACC = 16, RS = 1;
  __device__ static int row0(int g, int lane) { return 8 * g + 4 * (lane / 32); }
  using frag_t = bf16x8;
  using acc_t = f32x16;
  using acc_e = float;
  __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<_Float16> {
  static constexpr int TM = 32, KPL = 8, TK = 16, NACC = 16, RS = 1;
  __device__ static int row0(int g, int lane) { return 8 * g + 4 * (lane / 32); }
  using frag_t = f16x8;
  using acc_t = f32x16;
  using acc_e = float;
  __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  static constexpr int TM = 32, KPL = 1, TK = 2, NACC = 16, RS = 1;
  __device__ static int row0(int g, int lane) { return 8 * g + 4 * (lane / 32); }
  using frag_t = float;
  using acc_t = f32x16;
  using acc_e = float;
  __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<double> {
  static constexpr int TM = 16, KPL = 1, TK = 4, NACC = 4, RS = 4;
  __device__ static int row0(int, int lane) { return lane / 16; }
  using frag_t = double;
  using acc_t = f64x4;
  using acc_e = double;
  __device__ static acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Tile configurations: block BM x BN, depth BK, WGM x WGN waves.
template <int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
  static constexpr int THREADS = 64 * WGM * WGN;
};
// 256 x 256 x 64 with 8 waves of 128 x 64 (8 MFMA tiles, 128 accumulators
// each): a 64 KB k-tile per block fetched by 512 threads.
using CfgBig16 = Cfg<256, 256, 64, 2, 4>;
using CfgSmall16 = Cfg<128, 128, 64, 2, 2>;
using CfgF32 = Cfg<128, 128, 32, 2, 2>;
using CfgF64 = Cfg<64, 64, 16, 2, 2>;

struct GemmCtl {
  DevState st;
  int check_done;   // return when the PCG done flag is set
  int check_conv;   // G1: reduce ||r||^2 partials and stop on convergence
  int nparts_rr;
  int scale_in;     // G1 (FP16 operands): scale r by s = 1e-3 sqrt(N M / ||r||^2)
  int64_t npix;     // N M of the problem (for the scale)
  int small_tiles = 0;  // host-side choice of the tile configuration (not read by kernels)
};

// Tile order.  Workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2: block b runs on XCD b % 8.  Blocks are renumbered so that
// each XCD owns a contiguous range of tiles, and that range is walked in
// groups of GM tile-rows so the tiles resident on one XCD at a time share a
// few A row-panels and B column-panels in that XCD's L2.
__device__ __forceinline__ void tile_coords(int bid, int ntm, int ntn, int GM, int& tm, int& tn) {
  const int total = ntm * ntn;
  int t = bid;
  if (total % 8 == 0) t = (bid % 8) * (total / 8) + bid / 8;
  const int per_group = GM * ntn;
  const int group = t / per_group;
  const int first = group * GM;
  const int gsz = (ntm - first) < GM ? (ntm - first) : GM;
  const int in = t % per_group;
  tm = first + in % gsz;
  tn = in / gsz;
}

// C[m][n] = sum_k A[m][k] B[n][k]; A is AT (converted to OT while staging),
// B is OT.  M, N multiples of BM, BN; K a multiple of BK.  LDS is
// double-buffered: the next k-tile is fetched into registers while the
// current one feeds the MFMAs, then written to the other buffer; one barrier
// per k-tile.
template <class OT, class AT, class C, class Epi>
__device__ __forceinline__ void gemm_body(const AT* __restrict__ A, int64_t lda,
                                          const OT* __restrict__ B, int64_t ldb, int64_t K, int ntm,
                                          int ntn, int GM, int bid, float ascale, const Epi& epi,
                                          const GemmCtl& ctl) {
  using F = Mfma<OT>;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, NT = C::THREADS;
  constexpr int TM = F::TM;
  constexpr int WM = BM / C::WGM, WN = BN / C::WGN;
  constexpr int FM = WM / TM, FN = WN / TM;
  constexpr int PAD = 16 / (int)sizeof(OT);
  constexpr int LDS_LD = BK + PAD;
  constexpr int CH = (sizeof(OT) <= 2) ? 8 : (16 / (int)sizeof(OT));  // staging chunk along K
  constexpr int A_CHUNKS = BM * BK / CH / NT;
  constexpr int B_CHUNKS = BN * BK / CH / NT;
  static_assert(A_CHUNKS * CH * NT == BM * BK, "A tile staging");
  static_assert(B_CHUNKS * CH * NT == BN * BK, "B tile staging");

  if (ctl.check_done && ctl.st.fl[FL_DONE]) return;
  if (ctl.check_conv || ctl.scale_in) {
    const double rr = reduce_slot<NT>(ctl.st, PR_RR, ctl.nparts_rr);
    if (ctl.check_conv) {
      const double thr = ctl.st.sc[SC_TOL2] * ctl.st.sc[SC_BB];
      if (bid == 0 && threadIdx.x == 0) ctl.st.sc[SC_RR] = rr;
      if (rr <= thr) {
        if (bid == 0 && threadIdx.x == 0) ctl.st.fl[FL_DONE] = 1;
        return;
      }
    }
    if (ctl.scale_in) {
      // FP16 range: unit-RMS input times 1e-3 keeps the spectral division's
      // amplification (up to 1 / lambda_min) below the FP16 maximum and the
      // high modes above its smallest normal number.
      const double sc = rr > 0.0 ? 1e-3 * sqrt((double)ctl.npix / rr) : 1.0;
      ascale = (float)sc;
      if (bid == 0 && threadIdx.x == 0) ctl.st.sc[SC_SCALE] = (double)ascale;
    }
  }

  __shared__ __attribute__((aligned(16))) OT As[2][BM * LDS_LD];
  __shared__ __attribute__((aligned(16))) OT Bs[2][BN * LDS_LD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  int tm, tn;
  tile_coords(bid, ntm, ntn, GM, tm, tn);
  const int64_t m0 = (int64_t)tm * BM;
  const int64_t n0 = (int64_t)tn * BN;

  typename F::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int e = 0; e < F::NACC; ++e) acc[a][b][e] = 0;

  AT ra[A_CHUNKS][CH];
  OT rb[B_CHUNKS][CH];

  auto load_tile = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < A_CHUNKS; ++c) {
      const int idx = tid + c * NT;
      const int row = idx / (BK / CH);
      const int kc = (idx % (BK / CH)) * CH;
      const AT* src = A + (m0 + row) * lda + k0 + kc;
#pragma unroll
      for (int e = 0; e < CH; ++e) ra[c][e] = src[e];
    }
#pragma unroll
    for (int c = 0; c < B_CHUNKS; ++c) {
      const int idx = tid + c * NT;
      const int row = idx / (BK / CH);
      const int kc = (idx % (BK / CH)) * CH;
      const OT* src = B + (n0 + row) * ldb + k0 + kc;
#pragma unroll
      for (int e = 0; e < CH; ++e) rb[c][e] = src[e];
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int c = 0; c < A_CHUNKS; ++c) {
      const int idx = tid + c * NT;
      const int row = idx / (BK / CH);
      const int kc = (idx % (BK / CH)) * CH;
      OT tmp[CH];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        if constexpr (std::is_same<OT, AT>::value)
          tmp[e] = ra[c][e];
        else
          tmp[e] = (OT)((float)ra[c][e] * ascale);
      }
#pragma unroll
      for (int e = 0; e < CH; ++e) As[buf][row * LDS_LD + kc + e] = tmp[e];
    }
#pragma unroll
    for (int c = 0; c < B_CHUNKS; ++c) {
      const int idx = tid + c * NT;
      const int row = idx / (BK / CH);
      const int kc = (idx % (BK / CH)) * CH;
#pragma unroll
      for (int e = 0; e < CH; ++e) Bs[buf][row * LDS_LD + kc + e] = rb[c][e];
    }
  };

  const int64_t nk = K / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) load_tile((kt + 1) * BK);
    const OT* as = As[buf];
    const OT* bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < BK / F::TK; ++ks) {
      typename F::frag_t fa[FM], fb[FN];
      const int kk = ks * F::TK + F::KPL * (lane / TM);
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int row = wm * WM + a * TM + (lane % TM);
        fa[a] = *reinterpret_cast<const typename F::frag_t*>(&as[row * LDS_LD + kk]);
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int row = wn * WN + b * TM + (lane % TM);
        fb[b] = *reinterpret_cast<const typename F::frag_t*>(&bs[row * LDS_LD + kk]);
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = F::mma(fa[a], fb[b], acc[a][b]);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: group g of lane l holds rows row0(g, l) + t RS (t = 0..3) of
  // column l % TM of each MFMA tile.
  typename Epi::Acc part;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int g = 0; g < F::NACC / 4; ++g) {
        const int64_t m = m0 + wm * WM + a * TM + F::row0(g, lane);
        const int64_t n = n0 + wn * WN + b * TM + (lane % TM);
        typename F::acc_e v[4] = {acc[a][b][4 * g], acc[a][b][4 * g + 1], acc[a][b][4 * g + 2],
                                  acc[a][b][4 * g + 3]};
        epi.template apply<F::RS>(m, n, v, part);
        // keep the epilogue's loads from being hoisted across tiles
        __builtin_amdgcn_sched_barrier(0);
      }
  epi.template finish<NT>(part, ctl.st, bid);
}

template <class OT, class AT, class C, class Epi>
__global__ __launch_bounds__(C::THREADS) void gemm_nt_kernel(const AT* __restrict__ A, int64_t lda,
                                                             const OT* __restrict__ B, int64_t ldb,
                                                             int64_t K, int ntm, int ntn, int GM,
                                                             float ascale, Epi epi, GemmCtl ctl) {
  gemm_body<OT, AT, C, Epi>(A, lda, B, ldb, K, ntm, ntn, GM, (int)blockIdx.x, ascale, epi, ctl);
}

// ---- epilogues ------------------------------------------------------------
struct NoAcc {};

// Transposed store: Ct[n][m + t RS] = v[t] (operand type).
template <class OT>
struct EpiStoreT {
  OT* C;
  int64_t ldc;
  using Acc = NoAcc;
  template <int RS, class V>
  __device__ __forceinline__ void apply(int64_t m, int64_t n, const V (&v)[4], Acc&) const {
    OT* d = C + n * ldc + m;
#pragma unroll
    for (int t = 0; t < 4; ++t) d[t * RS] = (OT)v[t];
  }
  template <int NT>
  __device__ __forceinline__ void finish(Acc&, const DevState&, int) const {}
};

// Direct store with the spectral division: C[m][n] = v / (eigM[m] + eigN[n]),
// zero at (0,0) and on padding (tables hold +inf there).
template <class OT>
struct EpiScale {
  OT* C;
  int64_t ldc;
  const double* eigM;  // rows of this product are the l (column) modes
  const double* eigN;  // columns are the k (row) modes
  int zero_origin = 1; // (m, n) = (0, 0) is the constant mode (set to zero)
  using Acc = NoAcc;
  template <int RS, class V>
  __device__ __forceinline__ void apply(int64_t m, int64_t n, const V (&v)[4], Acc&) const {
    const double en = eigN[n];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t mm = m + t * RS;
      const double lam = eigM[mm] + en;
      const double f = (zero_origin && mm == 0 && n == 0) ? 0.0 : 1.0 / lam;
      C[mm * ldc + n] = (OT)((double)v[t] * f);
    }
  }
  template <int NT>
  __device__ __forceinline__ void finish(Acc&, const DevState&, int) const {}
};

// Final product, direct store: z = v * zscale (divided by the device-side
// input scale when given); the dot products follow in zdots_kernel.
template <class T>
struct EpiStoreZ {
  T* z;
  int64_t ldc;
  double zscale;
  const double* dscale;
  using Acc = NoAcc;
  template <int RS, class V>
  __device__ __forceinline__ void apply(int64_t m, int64_t n, const V (&v)[4], Acc&) const {
    const double zs = dscale ? zscale / *dscale : zscale;
#pragma unroll
    for (int t = 0; t < 4; ++t) z[(m + t * RS) * ldc + n] = (T)((double)v[t] * zs);
  }
  template <int NT>
  __device__ __forceinline__ void finish(Acc&, const DevState&, int) const {}
};

// z.r, z.q and sum z in one pass (FP64 partials), after the last product.
template <class T>
__device__ __forceinline__ void zdots_body(const T* z, const T* r, const T* q, int64_t n,
                                           const DevState& st, int lb, int nb) {
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t n4 = n / 4;
  for (int64_t k = (int64_t)lb * kThreads + threadIdx.x; k < n4; k += (int64_t)nb * kThreads) {
    const int64_t o = 4 * k;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double zd = (double)z[o + e];
      acc[0] += zd * (double)r[o + e];
      if (q) acc[1] += zd * (double)q[o + e];
      acc[2] += zd;
    }
  }
  const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
  write_partials<3>(st, slots, acc, lb);
}

template <class T>
__global__ __launch_bounds__(kThreads) void zdots_kernel(const T* z, const T* r, const T* q,
                                                         int64_t n, DevState st, int check_done) {
  if (check_done && st.fl[FL_DONE]) return;
  zdots_body<T>(z, r, q, n, st, (int)blockIdx.x, (int)gridDim.x);
}

// Final product: z (vector type T), partial sums of z.r, z.q, sum z.
template <class T>
struct EpiFinal {
  T* z;
  const T* r;
  const T* q;  // nullable
  int64_t ldc;
  double zscale;
  const double* dscale;  // nullable: divide by the device-side input scale
  struct Acc {
    double zr = 0.0, zq = 0.0, zs = 0.0;
  };
  template <int RS, class V>
  __device__ __forceinline__ void apply(int64_t m, int64_t n, const V (&v)[4], Acc& acc) const {
    const double zs = dscale ? zscale / *dscale : zscale;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t o = (m + t * RS) * ldc + n;
      const T zt = (T)((double)v[t] * zs);
      z[o] = zt;
      const double zd = (double)zt;
      acc.zr += zd * (double)r[o];
      if (q) acc.zq += zd * (double)q[o];
      acc.zs += zd;
    }
  }
  template <int NT>
  __device__ __forceinline__ void finish(Acc& acc, const DevState& st, int lb) const {
    double v[3] = {acc.zr, acc.zq, acc.zs};
    const int slots[3] = {PR_ZR, PR_ZQ, PR_ZS};
    write_partials<3, NT>(st, slots, v, lb);
  }
};

template <class OT>
struct CfgFor {
  using type = CfgSmall16;
};
template <>
struct CfgFor<float> {
  using type = CfgF32;
};
template <>
struct CfgFor<double> {
  using type = CfgF64;
};

// Launch one product with the largest configuration whose tiles divide the
// problem; returns the number of blocks (partials of the final epilogue).
template <class OT, class AT, class Epi, bool kBig = true>
static int gemm(const AT* A, int64_t lda, const OT* B, int64_t ldb, int64_t Mg, int64_t Ng,
                int64_t K, float ascale, const Epi& epi, const GemmCtl& ctl, hipStream_t s) {
  if constexpr (sizeof(OT) == 2 && kBig) {
    using CB = CfgBig16;
    if (!ctl.small_tiles && Mg % CB::BM == 0 && Ng % CB::BN == 0 && K % CB::BK == 0) {
      const int ntm = (int)(Mg / CB::BM), ntn = (int)(Ng / CB::BN);
      hipLaunchKernelGGL((gemm_nt_kernel<OT, AT, CB, Epi>), dim3(ntm * ntn), dim3(CB::THREADS), 0,
                         s, A, lda, B, ldb, K, ntm, ntn, 4, ascale, epi, ctl);
      return ntm * ntn;
    }
  }
  using CS = typename CfgFor<OT>::type;
  const int ntm = (int)(Mg / CS::BM), ntn = (int)(Ng / CS::BN);
  hipLaunchKernelGGL((gemm_nt_kernel<OT, AT, CS, Epi>), dim3(ntm * ntn), dim3(CS::THREADS), 0, s,
                     A, lda, B, ldb, K, ntm, ntn, 8, ascale, epi, ctl);
  return ntm * ntn;
}

template <class OT, class T>
static int precond_impl(const PrecondArgs& a, hipStream_t s) {
  const int64_t Np = a.Np, Mp = a.Mp;
  const OT* PN = static_cast<const OT*>(a.PN);
  const OT* PNt = static_cast<const OT*>(a.PNt);
  const OT* PM = static_cast<const OT*>(a.PM);
  const OT* PMt = static_cast<const OT*>(a.PMt);
  OT* T1 = static_cast<OT*>(a.T1);
  OT* T2 = static_cast<OT*>(a.T2);
  OT* T3 = static_cast<OT*>(a.T3);
  const T* r = static_cast<const T*>(a.r);
  const int f16 = std::is_same<OT, _Float16>::value ? 1 : 0;
  GemmCtl c1{a.st, 1, a.check_conv, a.nparts_rr, f16, a.N * a.M, a.small_tiles};
  GemmCtl cn{a.st, 1, 0, 0, 0, 0, a.small_tiles};
  LaunchLog* L = a.log;
  log_start(L, s);
  // G1: T1^T = (r P_M)^T
  gemm<OT, T>(r, Mp, PMt, Mp, Np, Mp, Mp, 1.0f, EpiStoreT<OT>{T1, Np}, c1, s);
  log_mark(L, IRLSU_LK_PRODUCT, s);
  // G2: T2^T = (P_N^T T1)^T ./ lambda
  gemm<OT, OT>(T1, Np, PNt, Np, Mp, Np, Np, 1.0f,
               EpiScale<OT>{T2, Np, static_cast<const double*>(a.eigM),
                            static_cast<const double*>(a.eigN)},
               cn, s);
  log_mark(L, IRLSU_LK_PRODUCT, s);
  // G3: T3 = (T2^T P_N^T)^T = P_N T2
  gemm<OT, OT>(T2, Np, PN, Np, Mp, Np, Np, 1.0f, EpiStoreT<OT>{T3, Mp}, cn, s);
  log_mark(L, IRLSU_LK_PRODUCT, s);
  // G4: z = T3 P_M^T.  16-bit operands: the 256 x 256 tile stores z only and
  // a light pass forms z.r, z.q, sum z (the fused epilogue does not fit
  // beside that tile's registers); FP32 / FP64 fuse the sums.
  if constexpr (sizeof(OT) == 2) {
    gemm<OT, OT>(T3, Mp, PM, Mp, Np, Mp, Mp, 1.0f,
                 EpiStoreZ<T>{static_cast<T*>(a.z), Mp, 1.0,
                              f16 ? a.st.sc + SC_SCALE : nullptr},
                 cn, s);
    log_mark(L, IRLSU_LK_PRODUCT, s);
    const int nb = elementwise_blocks(Np * Mp);
    hipLaunchKernelGGL(zdots_kernel<T>, dim3(nb), dim3(kThreads), 0, s, static_cast<const T*>(a.z),
                       r, static_cast<const T*>(a.q), Np * Mp, a.st, 1);
    log_mark(L, IRLSU_LK_DOTS, s);
    return nb;
  } else {
    const int nb = gemm<OT, OT>(T3, Mp, PM, Mp, Np, Mp, Mp, 1.0f,
                                EpiFinal<T>{static_cast<T*>(a.z), r, static_cast<const T*>(a.q), Mp,
                                            1.0, nullptr},
                                cn, s);
    log_mark(L, IRLSU_LK_PRODUCT, s);
    return nb;
  }
}

// Folded form: the same map with every dense product split into its even
// and odd halves (half the MFMA work); see fold.hip for the identities.
template <class OT, class T>
static int precond_folded_impl(const PrecondArgs& a, hipStream_t s) {
  const int64_t N = a.N, M = a.M, Np = a.Np, Mp = a.Mp, hN = a.hNp, hM = a.hMp;
  const int64_t wN = 2 * hN, wM = 2 * hM;  // folded widths
  const OT* PeN = static_cast<const OT*>(a.PeN);
  const OT* PeNt = static_cast<const OT*>(a.PeNt);
  const OT* PoN = static_cast<const OT*>(a.PoN);
  const OT* PoNt = static_cast<const OT*>(a.PoNt);
  const OT* PeM = static_cast<const OT*>(a.PeM);
  const OT* PeMt = static_cast<const OT*>(a.PeMt);
  const OT* PoM = static_cast<const OT*>(a.PoM);
  const OT* PoMt = static_cast<const OT*>(a.PoMt);
  const double* eN = static_cast<const double*>(a.eigNf);
  const double* eM = static_cast<const double*>(a.eigMf);
  OT* X1 = static_cast<OT*>(a.T1);
  OT* X2 = static_cast<OT*>(a.T2);
  T* ZEO = static_cast<T*>(a.ZEO);
  const T* r = static_cast<const T*>(a.r);
  const int f16 = std::is_same<OT, _Float16>::value ? 1 : 0;
  const int32_t* done = a.st.fl + FL_DONE;
  GemmCtl cn{a.st, 1, 0, 0, 0, 0, a.small_tiles};
  LaunchLog* L = a.log;
  auto prod = [&]() { log_mark(L, IRLSU_LK_PRODUCT, s); };
  auto pass = [&]() { log_mark(L, IRLSU_LK_BUTTERFLY, s); };
  log_start(L, s);
  launch_fold_prologue(a.st, a.nparts_rr, a.check_conv, f16, N * M, s);
  log_mark(L, IRLSU_LK_PROLOGUE, s);
  // S = [r_j + r_{M-1-j} | r_j - r_{M-1-j}]           (Np x wM)
  launch_fold_rows<T, OT>(r, Mp, M, N, Np, X1, hM, f16 ? a.st.sc + SC_SCALE : nullptr, done, s);
  pass();
  // T1^T: even / odd column modes, transposed stores     (wM x Np)
  gemm<OT, OT>(X1, wM, PeMt, hM, Np, hM, hM, 1.0f, EpiStoreT<OT>{X2, Np}, cn, s);
  prod();
  gemm<OT, OT>(X1 + hM, wM, PoMt, hM, Np, hM, hM, 1.0f, EpiStoreT<OT>{X2 + hM * Np, Np}, cn, s);
  prod();
  // fold the rows index of T1^T                           (wM x wN)
  launch_fold_rows<OT, OT>(X2, Np, N, wM, wM, X1, hN, nullptr, done, s);
  pass();
  // T2^T = (P_N^T T1)^T ./ lambda: even / odd row modes   (wM x wN)
  gemm<OT, OT>(X1, wN, PeNt, hN, wM, hN, hN, 1.0f, EpiScale<OT>{X2, wN, eM, eN, 1}, cn, s);
  prod();
  gemm<OT, OT>(X1 + hN, wN, PoNt, hN, wM, hN, hN, 1.0f, EpiScale<OT>{X2 + hN, wN, eM, eN + hN, 0},
               cn, s);
  prod();
  // inverse along rows: E and O stacked                   (wN x wM)
  gemm<OT, OT>(X2, wN, PeN, hN, wM, hN, hN, 1.0f, EpiStoreT<OT>{X1, wM}, cn, s);
  prod();
  gemm<OT, OT>(X2 + hN, wN, PoN, hN, wM, hN, hN, 1.0f, EpiStoreT<OT>{X1 + hN * wM, wM}, cn, s);
  prod();
  // T3 rows i, N-1-i = E +- O                              (Np x wM)
  launch_unfold_rows<OT>(X1, wM, N, hN, Np, X2, done, s);
  pass();
  // inverse along columns: zE | zO                         (Np x wM, vector type)
  gemm<OT, OT>(X2, wM, PeM, hM, Np, hM, hM, 1.0f, EpiStoreZ<T>{ZEO, wM, 1.0, nullptr}, cn, s);
  prod();
  gemm<OT, OT>(X2 + hM, wM, PoM, hM, Np, hM, hM, 1.0f, EpiStoreZ<T>{ZEO + hM, wM, 1.0, nullptr}, cn,
               s);
  prod();
  // z = zE +- zO (undoing the FP16 scale), z.r, z.q, sum z
  const int nb = launch_unfold_cols_dots<T>(ZEO, hM, N, M, Np, Mp, static_cast<T*>(a.z), r,
                                            static_cast<const T*>(a.q), 1.0,
                                            f16 ? a.st.sc + SC_SCALE : nullptr, a.st, s);
  log_mark(L, IRLSU_LK_DOTS, s);
  return nb;
}

int launch_precond(const PrecondArgs& a, hipStream_t s) {
  if (a.fast) return launch_precond_fast(a, s);
  if (a.folded) {
    switch (a.kind) {
      case OK_F64: return precond_folded_impl<double, double>(a, s);
      case OK_F32: return precond_folded_impl<float, float>(a, s);
      case OK_BF16: return precond_folded_impl<__bf16, float>(a, s);
      case OK_F16: return precond_folded_impl<_Float16, float>(a, s);
    }
  }
  switch (a.kind) {
    case OK_F64: return precond_impl<double, double>(a, s);
    case OK_F32: return precond_impl<float, float>(a, s);
    case OK_BF16: return precond_impl<__bf16, float>(a, s);
    case OK_F16: return precond_impl<_Float16, float>(a, s);
  }
  return 0;
}

// ---- grouped products over the tiles of a batch ------------------------
// The configuration of each product is fixed per launch: tiles are padded to
// multiples of 256, so 16-bit operands use the 256 x 256 tile and FP32
// operands the 128 x 128 one throughout.  Tiles in the fast form have no
// blocks here (their preconditioner runs its own passes).
template <class OT, int G>
struct BatchCfg {
  using type = CfgBig16;
};
template <int G>
struct BatchCfg<float, G> {
  using type = CfgF32;
};

template <class OT>
constexpr int batch_threads() {
  return BatchCfg<OT, 1>::type::THREADS;
}

template <class OT, class T, int G>
__global__ __launch_bounds__(batch_threads<OT>()) void gemm_batched_kernel(
    const BatchTile<T>* tiles, const int32_t* start, int ntiles, int check_conv) {
  using C = typename BatchCfg<OT, G>::type;
  const int t = find_tile(start, ntiles, (int)blockIdx.x);
  const BatchTile<T>& bt = tiles[t];
  const int bid = (int)blockIdx.x - start[t];
  const int64_t Np = bt.Np, Mp = bt.ld;
  constexpr int f16 = std::is_same<OT, _Float16>::value ? 1 : 0;
  GemmCtl ctl{bt.st, 1, G == 1 ? check_conv : 0, bt.st_nblk, G == 1 ? f16 : 0, bt.N * bt.M};
  if constexpr (G == 1) {
    gemm_body<OT, T, C>(bt.r, Mp, static_cast<const OT*>(bt.PMt), Mp, Mp, (int)(Np / C::BM),
                        (int)(Mp / C::BN), 4, bid, 1.0f,
                        EpiStoreT<OT>{static_cast<OT*>(bt.T1), Np}, ctl);
  } else if constexpr (G == 2) {
    gemm_body<OT, OT, C>(static_cast<const OT*>(bt.T1), Np, static_cast<const OT*>(bt.PNt), Np, Np,
                         (int)(Mp / C::BM), (int)(Np / C::BN), 4, bid, 1.0f,
                         EpiScale<OT>{static_cast<OT*>(bt.T2), Np, bt.eigM, bt.eigN}, ctl);
  } else if constexpr (G == 3) {
    gemm_body<OT, OT, C>(static_cast<const OT*>(bt.T2), Np, static_cast<const OT*>(bt.PN), Np, Np,
                         (int)(Mp / C::BM), (int)(Np / C::BN), 4, bid, 1.0f,
                         EpiStoreT<OT>{static_cast<OT*>(bt.T3), Mp}, ctl);
  } else {
    gemm_body<OT, OT, C>(static_cast<const OT*>(bt.T3), Mp, static_cast<const OT*>(bt.PM), Mp, Mp,
                         (int)(Np / C::BM), (int)(Mp / C::BN), 4, bid, 1.0f,
                         EpiStoreZ<T>{bt.z, Mp, 1.0, f16 ? bt.st.sc + SC_SCALE : nullptr}, ctl);
  }
}

void precond_blocks(int kind, int64_t Np, int64_t Mp, int out[4]) {
  const int64_t B = kind == OK_F32 ? CfgF32::BM : CfgBig16::BM;
  out[0] = (int)((Np / B) * (Mp / B));
  out[1] = (int)((Mp / B) * (Np / B));
  out[2] = out[1];
  out[3] = out[0];
}

// Grouped z.r / z.q / sum z over a batch: each tile uses its stencil block
// count (st_nblk), which is also its g4_nparts.
template <class T>
__global__ __launch_bounds__(kThreads) void zdots_batched_kernel(const BatchTile<T>* tiles,
                                                                 const int32_t* start, int ntiles) {
  const int t = find_tile(start, ntiles, (int)blockIdx.x);
  const BatchTile<T>& bt = tiles[t];
  if (bt.fast || bt.st.fl[FL_DONE]) return;
  zdots_body<T>(bt.z, bt.r, bt.flexible_q ? bt.q : nullptr, bt.Np * bt.ld, bt.st,
                (int)blockIdx.x - start[t], bt.st_nblk);
}

template <class OT>
static void precond_batched_impl(const BatchTile<float>* tiles, const int32_t* starts, int ntiles,
                                 const int* totals, int check_conv, hipStream_t s) {
  const int n1 = ntiles + 1;
  constexpr int TH = batch_threads<OT>();
  hipLaunchKernelGGL((gemm_batched_kernel<OT, float, 1>), dim3(totals[0]), dim3(TH), 0, s, tiles,
                     starts, ntiles, check_conv);
  hipLaunchKernelGGL((gemm_batched_kernel<OT, float, 2>), dim3(totals[1]), dim3(TH), 0, s, tiles,
                     starts + n1, ntiles, 0);
  hipLaunchKernelGGL((gemm_batched_kernel<OT, float, 3>), dim3(totals[2]), dim3(TH), 0, s, tiles,
                     starts + 2 * n1, ntiles, 0);
  hipLaunchKernelGGL((gemm_batched_kernel<OT, float, 4>), dim3(totals[3]), dim3(TH), 0, s, tiles,
                     starts + 3 * n1, ntiles, 0);
}

void launch_precond_batched(int kind, const void* tiles, const int32_t* starts, int ntiles,
                            const int* totals, int check_conv, const int32_t* st_start,
                            int st_total, hipStream_t s) {
  const BatchTile<float>* t = static_cast<const BatchTile<float>*>(tiles);
  if (totals[0] > 0) {  // no grouped products when every tile is in the fast form
    if (kind == OK_F16)
      precond_batched_impl<_Float16>(t, starts, ntiles, totals, check_conv, s);
    else if (kind == OK_F32)
      precond_batched_impl<float>(t, starts, ntiles, totals, check_conv, s);
    else
      precond_batched_impl<__bf16>(t, starts, ntiles, totals, check_conv, s);
  }
  hipLaunchKernelGGL(zdots_batched_kernel<float>, dim3(st_total), dim3(kThreads), 0, s, t, st_start,
                     ntiles);
}

// ---- basis tables ------------------------------------------------------
// P[i][k] = c_k cos(pi k (2i+1) / (2n)), c_0 = sqrt(1/n), c_k = sqrt(2/n);
// the angle index k (2i+1) is reduced modulo 4n exactly in integers.
// eig[k] = 2 - 2 cos(pi k / n) = 4 sin^2(pi k / 2n) (no cancellation), +inf
// on padding so that the spectral division yields zero there.
template <class OT>
__global__ __launch_bounds__(kThreads) void basis_kernel(int64_t n, int64_t npad, OT* P, OT* Pt,
                                                        double* eig) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (k >= npad) return;
  double v = 0.0;
  if (i < n && k < n) {
    const int64_t idx = (k * (2 * i + 1)) % (4 * n);
    const double ang = 3.141592653589793 * (double)idx / (double)(2 * n);
    v = cos(ang) * (k == 0 ? sqrt(1.0 / (double)n) : sqrt(2.0 / (double)n));
  }
  P[i * npad + k] = (OT)v;
  Pt[k * npad + i] = (OT)v;
  if (i == 0) {
    if (k < n) {
      const double sn = sin(3.141592653589793 * (double)k / (double)(2 * n));
      eig[k] = 4.0 * sn * sn;
    } else {
      eig[k] = __builtin_inf();
    }
  }
}

void launch_basis(int kind, int64_t n, int64_t npad, void* P, void* Pt, void* eig, hipStream_t s) {
  const dim3 grid((unsigned)((npad + kThreads - 1) / kThreads), (unsigned)npad);
  double* e = static_cast<double*>(eig);
  switch (kind) {
    case OK_F64:
      hipLaunchKernelGGL(basis_kernel<double>, grid, dim3(kThreads), 0, s, n, npad,
                         static_cast<double*>(P), static_cast<double*>(Pt), e);
      break;
    case OK_F32:
      hipLaunchKernelGGL(basis_kernel<float>, grid, dim3(kThreads), 0, s, n, npad,
                         static_cast<float*>(P), static_cast<float*>(Pt), e);
      break;
    case OK_BF16:
      hipLaunchKernelGGL(basis_kernel<__bf16>, grid, dim3(kThreads), 0, s, n, npad,
                         static_cast<__bf16*>(P), static_cast<__bf16*>(Pt), e);
      break;
    case OK_F16:
      hipLaunchKernelGGL(basis_kernel<_Float16>, grid, dim3(kThreads), 0, s, n, npad,
                         static_cast<_Float16*>(P), static_cast<_Float16*>(Pt), e);
      break;
  }
}

}  // namespace irlsu
