// Complex arithmetic, small DFTs in registers and 16-byte streaming
// accesses shared by the fast-form passes (power-of-two sides in fct.hip,
// sides with factors 2, 3 and 5 in fctg.hip).
#pragma once
#include <cstdint>
#include <type_traits>

#include <hip/hip_runtime.h>

namespace irlsu {

template <class CT>
struct Cx {
  CT x, y;
};

template <class CT>
__device__ __forceinline__ Cx<CT> cadd(Cx<CT> a, Cx<CT> b) {
  return {a.x + b.x, a.y + b.y};
}
template <class CT>
__device__ __forceinline__ Cx<CT> csub(Cx<CT> a, Cx<CT> b) {
  return {a.x - b.x, a.y - b.y};
}
template <class CT>
__device__ __forceinline__ Cx<CT> cmul(Cx<CT> a, Cx<CT> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <class CT>
__device__ __forceinline__ Cx<CT> cmulc(Cx<CT> a, Cx<CT> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <class CT>
__device__ __forceinline__ Cx<CT> conjg(Cx<CT> a) {
  return {a.x, -a.y};
}
// -i a
template <class CT>
__device__ __forceinline__ Cx<CT> mul_mi(Cx<CT> a) {
  return {a.y, -a.x};
}
// i a
template <class CT>
__device__ __forceinline__ Cx<CT> mul_i(Cx<CT> a) {
  return {-a.y, a.x};
}
template <class CT>
__device__ __forceinline__ Cx<CT> cscale(Cx<CT> a, CT s) {
  return {a.x * s, a.y * s};
}
// 1 / x: correctly rounded in FP64; in FP32 the hardware reciprocal (1 ulp),
// well inside the FP32 transform's own rounding
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Calls f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---- small forward DFTs in registers (natural order in and out) ----------
template <class CT>
__device__ __forceinline__ void dft4(Cx<CT>& a0, Cx<CT>& a1, Cx<CT>& a2, Cx<CT>& a3) {
  const Cx<CT> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// e^{-2 pi i j / 16}, j = 0..15 (the twiddles of the 4 x 4 split)
template <class CT>
__device__ __forceinline__ Cx<CT> w16(int j) {
  // cos(2 pi j / 16) for j = 0..15; sin is the cosine a quarter turn back
  constexpr double c[16] = {1.0,
                            0.92387953251128675613,
                            0.70710678118654752440,
                            0.38268343236508977173,
                            0.0,
                            -0.38268343236508977173,
                            -0.70710678118654752440,
                            -0.92387953251128675613,
                            -1.0,
                            -0.92387953251128675613,
                            -0.70710678118654752440,
                            -0.38268343236508977173,
                            0.0,
                            0.38268343236508977173,
                            0.70710678118654752440,
                            0.92387953251128675613};
  return {(CT)c[j & 15], (CT)(-c[(j + 12) & 15])};
}

// a * e^{-2 pi i J / 16} for a compile-time J: quarter turns by swaps and
// sign changes, odd eighth turns by one add and one multiply per part, the
// rest by a complex product with the constant.
template <class CT, int J>
__device__ __forceinline__ Cx<CT> mul_w16(Cx<CT> a) {
  constexpr int j = J & 15;
  constexpr CT h = (CT)0.70710678118654752440;
  if constexpr (j == 0) {
    return a;
  } else if constexpr (j == 4) {
    return mul_mi(a);
  } else if constexpr (j == 8) {
    return {-a.x, -a.y};
  } else if constexpr (j == 12) {
    return mul_i(a);
  } else if constexpr (j == 2) {   // h (1 - i)
    return {(a.x + a.y) * h, (a.y - a.x) * h};
  } else if constexpr (j == 6) {   // h (-1 - i)
    return {(a.y - a.x) * h, -(a.x + a.y) * h};
  } else if constexpr (j == 10) {  // h (-1 + i)
    return {-(a.x + a.y) * h, (a.x - a.y) * h};
  } else if constexpr (j == 14) {  // h (1 + i)
    return {(a.x - a.y) * h, (a.x + a.y) * h};
  } else {
    return cmul(a, w16<CT>(j));
  }
}

template <class CT, int R>
__device__ __forceinline__ void dft(Cx<CT> (&a)[R]) {
  if constexpr (R == 2) {
    const Cx<CT> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (R == 4) {
    dft4(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    // n = 4 n1 + n2, k = k1 + 2 k2: length-2 DFTs over n1, twiddle
    // e^{-2 pi i n2 k1 / 8}, length-4 DFTs over n2
    Cx<CT> b0[4], b1[4];
    static_for<0, 4>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      b0[n2] = cadd(a[n2], a[4 + n2]);
      b1[n2] = mul_w16<CT, 2 * n2>(csub(a[n2], a[4 + n2]));
    });
    dft4(b0[0], b0[1], b0[2], b0[3]);
    dft4(b1[0], b1[1], b1[2], b1[3]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      a[2 * k2] = b0[k2];
      a[1 + 2 * k2] = b1[k2];
    }
  } else {
    static_assert(R == 16, "radix");
    // n = 4 n1 + n2, k = k1 + 4 k2
    Cx<CT> b[4][4];
    static_for<0, 4>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      Cx<CT> c0 = a[n2], c1 = a[4 + n2], c2 = a[8 + n2], c3 = a[12 + n2];
      dft4(c0, c1, c2, c3);
      b[0][n2] = c0;
      b[1][n2] = mul_w16<CT, n2>(c1);
      b[2][n2] = mul_w16<CT, 2 * n2>(c2);
      b[3][n2] = mul_w16<CT, 3 * n2>(c3);
    });
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      dft4(b[k1][0], b[k1][1], b[k1][2], b[k1][3]);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = b[k1][k2];
    }
  }
}

// e^{-2 pi i / 3} and e^{-2 pi i / 5}: small DFTs of radix 3 and 5 written out
// from the definition X_k = sum_m a_m w^{m k}, pairing a_m with a_{R-m}
// (w^{R-m} = conj w^m): the pair's sum meets the cosines, its difference the
// sines.
template <class CT>
__device__ __forceinline__ void dft3(Cx<CT>& a0, Cx<CT>& a1, Cx<CT>& a2) {
  const CT s = (CT)0.86602540378443864676;   // sin(2 pi / 3)
  const Cx<CT> b = cadd(a1, a2), d = csub(a1, a2);
  const Cx<CT> m = {a0.x - (CT)0.5 * b.x, a0.y - (CT)0.5 * b.y};
  const Cx<CT> t = {d.y * s, -d.x * s};      // -i s d
  a0 = cadd(a0, b);
  a1 = cadd(m, t);
  a2 = csub(m, t);
}

template <class CT>
__device__ __forceinline__ void dft5(Cx<CT> (&a)[5]) {
  const CT c1 = (CT)0.30901699437494742410, c2 = (CT)-0.80901699437494742410;  // cos 2pi/5, 4pi/5
  const CT s1 = (CT)0.95105651629515357212, s2 = (CT)0.58778525229247312917;   // sin 2pi/5, 4pi/5
  const Cx<CT> b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
  const Cx<CT> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
  const Cx<CT> m1 = {a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y};
  const Cx<CT> m2 = {a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y};
  // -i (s1 d1 + s2 d2) and -i (s2 d1 - s1 d2)
  const Cx<CT> e1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
  const Cx<CT> e2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
  const Cx<CT> t1 = mul_mi(e1), t2 = mul_mi(e2);
  a[0] = {a[0].x + b1.x + b2.x, a[0].y + b1.y + b2.y};
  a[1] = cadd(m1, t1);
  a[4] = csub(m1, t1);
  a[2] = cadd(m2, t2);
  a[3] = csub(m2, t2);
}

// Everything the column pass's pair step k (0 <= k <= h/2) of a side of
// length n = 2h reads, in one 16-byte aligned record: e^{-i pi k/(2n)},
// e^{-i pi (h-k)/(2n)}, e^{-2 pi i k/n} and the eigenvalues 4 sin^2(pi j/2n)
// at j = k, n-k (0 for k = 0), h-k, h+k times escale; each value rounded
// once from FP64.
template <class CT>
struct alignas(16) PairTw {
  Cx<CT> q, qp, n;
  CT e[6];
};

// Start of the pair records in a side's table, in CT elements: after 3h + 2
// complex entries (6h + 4 CT, so 16-byte aligned).
__host__ __device__ inline int64_t pair_table_offset(int64_t h) { return 2 * (3 * h + 2); }

template <class CT>
__device__ __forceinline__ void pair_tw_fill(PairTw<CT>* out, int64_t k, int64_t h,
                                             double escale) {
  const double n = 2.0 * (double)h;
  double s, c;
  PairTw<CT> t;
  sincospi(0.5 * (double)k / n, &s, &c);
  t.q = {(CT)c, (CT)(-s)};
  sincospi(0.5 * (double)(h - k) / n, &s, &c);
  t.qp = {(CT)c, (CT)(-s)};
  sincospi(2.0 * (double)k / n, &s, &c);
  t.n = {(CT)c, (CT)(-s)};
  const int64_t j[4] = {k, 2 * h - k, h - k, h + k};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double sv = sinpi(0.5 * (double)j[i] / n);
    t.e[i] = (i == 1 && k == 0) ? (CT)0 : (CT)(4.0 * sv * sv * escale);
  }
  t.e[4] = t.e[5] = (CT)0;
  *out = t;
}

// ---- DCT pair steps (one length-n DCT through an FFT of h = n/2 points) --
// Forward post-processing of pair k (0 <= k <= h/2): twice c_k and c_{h-k}
// from W_k and W_{h-k}, with tq = e^{-i pi k/(2n)}, tqp = e^{-i pi (h-k)/(2n)}
// and tn = e^{-2 pi i k/n}.  With E = W_k + conj W_{h-k} and O = -i (W_k -
// conj W_{h-k}), index h-k has conj E and conj O, and e^{-2 pi i (h-k)/n} =
// -conj tn: one product P = tn O gives V_k = E + P and V_{h-k} = conj(E - P).
template <class CT>
__device__ __forceinline__ void post_core(Cx<CT> wa, Cx<CT> wb, Cx<CT> tq, Cx<CT> tqp, Cx<CT> tn,
                                          Cx<CT>& ck, Cx<CT>& cp) {
  const Cx<CT> E = {wa.x + wb.x, wa.y - wb.y};
  const Cx<CT> O = {wa.y + wb.y, wb.x - wa.x};
  const Cx<CT> P = cmul(tn, O);
  ck = cmul(tq, cadd(E, P));
  cp = cmul(tqp, {E.x - P.x, P.y - E.y});
}

// Inverse pre-processing of pair k: from c_k = Xt_k - i Xt_{n-k} and
// c_{h-k}, the (conjugated) FFT inputs twice W_k (sk) and W_{h-k} (sp).
// With v = conj(tq) c at k and at h-k, E = v_k + conj v_{h-k} and O = (v_k -
// conj v_{h-k}) conj tn; index h-k has conj E and conj O (the identities of
// post_core), so sk = conj(E + i O) and sp = E - i O.
template <class CT>
__device__ __forceinline__ void pre_core(Cx<CT> ck, Cx<CT> cp, Cx<CT> tq, Cx<CT> tqp, Cx<CT> tn,
                                         Cx<CT>& sk, Cx<CT>& sp) {
  const Cx<CT> vk = cmulc(ck, tq);
  const Cx<CT> vp = cmulc(cp, tqp);
  const Cx<CT> E = {vk.x + vp.x, vk.y - vp.y};
  const Cx<CT> O = cmulc({vk.x - vp.x, vk.y + vp.y}, tn);
  sk = {E.x - O.y, -E.y - O.x};
  sp = {E.x + O.y, E.y - O.x};
}

template <class T>
struct Vec16 {
  static constexpr int W = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

// 16-byte streaming accesses (non-temporal hint) for data a pass reads or
// writes once
template <class V, class T>
__device__ __forceinline__ V ld_nt(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
}
template <class V, class T>
__device__ __forceinline__ void st_nt(T* p, const V& v) {
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

}  // namespace irlsu
