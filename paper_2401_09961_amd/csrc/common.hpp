// Shared definitions of the irlsu HIP kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "irlsu.h"

namespace irlsu {

constexpr int kThreads = 256;          // every kernel runs 4 wave64s per block
constexpr int kMaxPartials = 262144;   // per-block partial sums per quantity (all tiles)
constexpr int kTilePad = 128;          // internal rows / row stride multiple
constexpr int64_t kMaxSide = 32768;    // largest N or M (2-D grids index rows in y)

// Slots of the per-plan device scalar array (double).
enum Scalar : int {
  SC_RHO = 0,      // [2] rho_l = r_l . z_l, double-buffered by iteration parity
  SC_ALPHA = 2,    // [2] alpha_l, double-buffered by parity
  SC_BETA = 4,
  SC_PQ = 5,
  SC_RR = 6,       // ||r||^2 of the last reduced residual
  SC_BB = 7,       // ||b||^2
  SC_L1 = 8,
  SC_H = 9,
  SC_MEAN = 10,
  SC_TOL2 = 11,    // pcg_rtol^2
  SC_ZSUM = 12,
  SC_SCALE = 13,   // FP16 preconditioner input scale
  SC_SOLD = 14,    // IRLS model at U^k with the previous weights
  SC_SNEW = 15,    // IRLS model at U^k with the new weights
  SC_INVL = 16,    // augmented form: 1 / L of Theorem 3
  SC_COUNT = 32
};

// Slots of the per-plan device flag array (int32).
enum Flag : int {
  FL_DONE = 0,     // PCG of the current IRLS iteration has stopped
  FL_ITERS = 1,    // PCG iterations performed
  FL_STATUS = 2,   // bit 0: breakdown
  FL_INPUT = 3,    // bit 0: non-finite input, bit 1: weight <= 0
  FL_GUARD = 4,    // augmented form: outcome of the sufficient-decrease guard
  FL_DPEND = 5,    // fast form: the iterate update of the iteration that
                   // converged is still owed by the row DCT-III pass
  FL_COUNT = 16
};

// Partial-sum slots: part[slot * kMaxPartials + block].
enum Part : int {
  PT_A = 0,        // first quantity of the producing kernel
  PT_B = 1,
  PT_C = 2,
  PT_D = 3,
  PT_COUNT = 4
};

// Quantities by slot for each producer:
//   weights:  A = sum C|r|, B = sum C h_eps(r), C = ||b||^2
//   residual/axpy: A = ||r||^2, B = sum r
//   stencil:  C = p . q            (kept apart from the residual slots)
//   precond:  D = z . r, and PT_Q_ZQ / PT_Q_ZS below
enum PartRole : int {
  PR_L1 = PT_A, PR_H = PT_B, PR_BB = PT_C,
  PR_RR = PT_A, PR_RSUM = PT_B,
  PR_PQ = PT_C,
  PR_ZR = PT_D,
};
constexpr int kPartSlots = 7;   // A..D plus precond's z.q and sum z
constexpr int PR_ZQ = 4;
constexpr int PR_ZS = 5;
constexpr int PR_AUX = 6;

// Device state of one problem (one image, or one tile of a batch): its
// scalars and flags, and its range [off, off + blocks) of every row of the
// shared partial-sum table.
struct DevState {
  double* sc = nullptr;    // SC_COUNT doubles
  int32_t* fl = nullptr;   // FL_COUNT ints
  double* part = nullptr;  // kPartSlots * kMaxPartials doubles (shared by all problems)
  int32_t off = 0;         // first partial index of this problem
  int32_t stride = 0;      // distance between two slots' rows; 0: kMaxPartials
};

// Row of partial sums of one slot for this problem: part[slot * stride + off ..].
__host__ __device__ __forceinline__ double* part_row(const DevState& st, int slot) {
  const size_t stride = st.stride > 0 ? (size_t)st.stride : (size_t)kMaxPartials;
  return st.part + (size_t)slot * stride + st.off;
}
inline double* part_row_host(const DevState& st, int slot) { return part_row(st, slot); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Deterministic block sum of NV doubles over NT threads; the result is
// returned in every thread.  Fixed shuffle tree inside each wave, then the
// waves summed in order.
template <int NV, int NT = kThreads>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[NV][NT / 64];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = wave_sum(v[k]);
    if (lane == 0) red[k][wid] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Reduce n partials of one slot in a fixed order; identical in every block.
// (Unrolled: the loads of eight partials are in flight together; the sum
// keeps its order.)
template <int NT = kThreads>
__device__ __forceinline__ double reduce_slot(const DevState& st, int slot, int n) {
  const double* p = part_row(st, slot);
  double s[1] = {0.0};
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += NT) s[0] += p[i];
  block_sum<1, NT>(s);
  return s[0];
}

__device__ __forceinline__ int linear_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

__device__ __forceinline__ int nblocks() {
  return gridDim.x * gridDim.y * gridDim.z;
}

// Block-reduce NV quantities and store them as partial number lb (the
// block's index within its problem).
template <int NV, int NT = kThreads>
__device__ __forceinline__ void write_partials(const DevState& st, const int (&slots)[NV],
                                               double (&v)[NV], int lb) {
  block_sum<NV, NT>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part_row(st, slots[k])[lb] = v[k];
  }
}

// Four consecutive elements, moved with 16-byte accesses (two for FP64).
template <class T>
struct V4 {
  T v[4];
};

template <class T>
__device__ __forceinline__ V4<T> ld4(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}

template <class T>
__device__ __forceinline__ void st4(T* p, const V4<T>& r) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(r.v[2], r.v[3]);
  }
}

// Streaming load (non-temporal hint): for data read once per pass.
template <class T>
__device__ __forceinline__ V4<T> ld4_nt(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 x = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p + 2));
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}

// Streaming store (non-temporal hint): for data written once per pass and
// not read again by the same kernel.
template <class T>
__device__ __forceinline__ void st4_nt(T* p, const V4<T>& r) {
  if constexpr (sizeof(T) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 v = {r.v[0], r.v[1], r.v[2], r.v[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p));
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 a = {r.v[0], r.v[1]}, b = {r.v[2], r.v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<d2*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<d2*>(p + 2));
  }
}

template <class T>
__device__ __forceinline__ V4<T> zero4() {
  V4<T> r;
  r.v[0] = r.v[1] = r.v[2] = r.v[3] = (T)0;
  return r;
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace irlsu
