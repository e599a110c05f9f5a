// Streaming bandwidth probes: the measured HBM ceilings that the kernels'
// achieved bandwidth is reported against (a plain copy, a read-only stream
// and a three-read / one-write stream, the operator's mix).  Each thread
// moves two 16-byte chunks per array per trip with non-temporal hints, over
// a grid-stride loop; the caller sweeps the grid size.
#include "kernels.hpp"

namespace irlsu {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int NR, int NW>
__global__ __launch_bounds__(kThreads) void stream_kernel(const f4* __restrict__ a,
                                                         const f4* __restrict__ b,
                                                         const f4* __restrict__ c,
                                                         f4* __restrict__ d, int64_t n16,
                                                         float* sink) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t i0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; i0 < n16; i0 += 2 * stride) {
    f4 x[2], y[2], z[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n16) {
        x[u] = __builtin_nontemporal_load(a + i);
        if (NR > 1) y[u] = __builtin_nontemporal_load(b + i);
        if (NR > 2) z[u] = __builtin_nontemporal_load(c + i);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n16) {
        f4 v = x[u];
        if (NR > 2) v = v + y[u] * z[u];
        else if (NR > 1) v = v + y[u];
        if (NW > 0) __builtin_nontemporal_store(v, d + i);
        else acc = acc + v;
      }
    }
  }
  // read-only stream: keep the loads live without writing the stream
  if (NW == 0 && acc.x == 1.2345e-30f && sink) sink[0] = acc.y + acc.z + acc.w;
}

// kind 0: copy (1 read, 1 write); 1: read only; 2: three reads, one write.
// Returns the mean milliseconds per launch over reps launches.
int launch_stream_probe(int kind, const void* a, const void* b, const void* c, void* d,
                        size_t bytes, int grid, int reps, float* ms, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const f4* fa = static_cast<const f4*>(a);
  const f4* fb = static_cast<const f4*>(b);
  const f4* fc = static_cast<const f4*>(c);
  f4* fd = static_cast<f4*>(d);
  float* sink = static_cast<float*>(d);
  auto launch = [&]() {
    switch (kind) {
      case 0: hipLaunchKernelGGL((stream_kernel<1, 1>), dim3(grid), dim3(kThreads), 0, s, fa, fb, fc, fd, n16, sink); break;
      case 1: hipLaunchKernelGGL((stream_kernel<1, 0>), dim3(grid), dim3(kThreads), 0, s, fa, fb, fc, fd, n16, sink); break;
      default: hipLaunchKernelGGL((stream_kernel<3, 1>), dim3(grid), dim3(kThreads), 0, s, fa, fb, fc, fd, n16, sink); break;
    }
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1;
  }
  launch();  // warm-up
  int rc = 0;
  if (hipEventRecord(e0, s) != hipSuccess) rc = -1;
  for (int r = 0; r < reps && rc == 0; ++r) launch();
  if (rc == 0 && hipEventRecord(e1, s) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -1;
  float t = 0.f;
  if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -1;
  if (rc == 0 && hipGetLastError() != hipSuccess) rc = -1;
  *ms = t / (float)reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace irlsu
