// Weighted 5-point operator q = D^T Omega D p on the image (the U block of the
// linear system of Proposition 1 after slack elimination; S^T S and T T^T of
// Appendix A are its unweighted form), fused with the CG direction update
// p = z + beta p (Algorithm 2) and the FP64 partial sum of p . q.
//
// Layout: row-major, ld columns.  A block owns 1024 columns and a band of
// rows; each of its four waves owns 256 of the columns (4 per lane, one
// 16-byte access per array per row for FP32) and walks the band top to
// bottom on its own, keeping the rows above / at / below the current one in
// registers.  The column halo comes from the neighbouring lanes by
// cross-lane shuffles; only the wave's two edge lanes read their outside
// neighbour from memory, so no wave waits for another (no barrier in the
// row loop).  The weights and halo of row i+1 and the p row i+2 are loaded
// before row i is computed, up to the last row the band needs.  The weights
// and q are streamed with non-temporal hints (on gfx950 that lifts a
// three-read / one-write stream from about 5.2 to 5.7 TB/s at 8192^2); p,
// which the preconditioner's last pass wrote just before with plain stores,
// is read with plain loads so that the last-level cache serves part of it
// (6% less time per PCG iteration at 8192^2, with the plain stores of the
// transposes and of p).  HBM traffic per
// pixel: p, Omega^v, Omega^h in, q out = 16 bytes (FP32; fused form z,
// p_old in and p out as well), plus the two halo rows per band.
#include "kernels.hpp"

namespace irlsu {

// CT: compute type (double in the residual mode, where u is FP64).
template <class T, int MODE>
struct StencilIO {
  using CT = typename std::conditional<MODE == ST_RESID, double, T>::type;
  const StencilArgs<T>& a;
  CT beta, zc;

  __device__ StencilIO(const StencilArgs<T>& a_, CT beta_, CT zc_) : a(a_), beta(beta_), zc(zc_) {}

  // p value of one pixel (scalar; used for the column halo).
  __device__ __forceinline__ CT p1(int64_t i, int64_t j) const {
    if (i < 0 || i >= a.Np || j < 0 || j >= a.ld) return (CT)0;
    const int64_t o = i * a.ld + j;
    if constexpr (MODE == ST_FUSED) {
      if (i >= a.N || j >= a.M) return (CT)0;
      return ((CT)a.z[o] - zc) + beta * (CT)a.p_in[o];
    } else if constexpr (MODE == ST_APPLY) {
      return (CT)a.p_in[o];
    } else {
      return (CT)a.u[o] + (a.d ? (CT)a.d[o] : (CT)0);
    }
  }

  // p values of 4 consecutive pixels (j multiple of 4, j < ld).
  __device__ __forceinline__ V4<CT> p4(int64_t i, int64_t j) const {
    V4<CT> r;
    if (i < 0 || i >= a.Np) {
      r.v[0] = r.v[1] = r.v[2] = r.v[3] = (CT)0;
      return r;
    }
    const int64_t o = i * a.ld + j;
    if constexpr (MODE == ST_FUSED) {
      const V4<T> z = ld4_nt(a.z + o);
      const V4<T> p = ld4_nt(a.p_in + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool valid = (i < a.N) && (j + e < a.M);
        r.v[e] = valid ? ((CT)z.v[e] - zc) + beta * (CT)p.v[e] : (CT)0;
      }
    } else if constexpr (MODE == ST_APPLY) {
      // a plain load: the direction was written just before by the
      // preconditioner's last pass and is partly in the last-level cache
      const V4<T> p = ld4(a.p_in + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) r.v[e] = (CT)p.v[e];
    } else {
      const V4<double> u = ld4_nt(a.u + o);
      const V4<T> d = a.d ? ld4_nt(a.d + o) : zero4<T>();
#pragma unroll
      for (int e = 0; e < 4; ++e) r.v[e] = (CT)u.v[e] + (CT)d.v[e];
    }
    return r;
  }
};

// Body shared by the single-image and the grouped (batched) launch: column
// block bx, row band by, block lb of its problem.
template <class T, int MODE>
__device__ __forceinline__ void stencil_body(const StencilArgs<T>& a, int bx, int by,
                                             int rows_per_block, int lb) {
  using IO = StencilIO<T, MODE>;
  using CT = typename IO::CT;
  if (a.check_done && a.st.fl[FL_DONE]) {
    // the row DCT-III pass before this launch paid the iterate update that
    // the converged iteration owed
    if (lb == 0 && threadIdx.x == 0 && a.st.fl[FL_DPEND]) a.st.fl[FL_DPEND] = 0;
    return;
  }

  CT beta = 0, zc = 0;
  if constexpr (MODE == ST_FUSED) {
    const double zr = reduce_slot(a.st, PR_ZR, a.nparts_prec);
    const double zs = reduce_slot(a.st, PR_ZS, a.nparts_prec);
    const double zq = reduce_slot(a.st, PR_ZQ, a.nparts_prec);
    const double rsum = reduce_slot(a.st, PR_RSUM, a.nparts_res);
    const double zcd = zs / ((double)a.N * (double)a.M);
    const double rho = zr - zcd * rsum;
    double b = 0.0;
    if (a.iter > 0) {
      const double rho_old = a.st.sc[SC_RHO + ((a.iter - 1) & 1)];
      if (a.flexible) {
        const double alpha_old = a.st.sc[SC_ALPHA + ((a.iter - 1) & 1)];
        b = -alpha_old * zq / rho_old;
      } else {
        b = rho / rho_old;
      }
    }
    if (lb == 0 && threadIdx.x == 0) {
      a.st.sc[SC_RHO + (a.iter & 1)] = rho;
      a.st.sc[SC_BETA] = b;
      a.st.sc[SC_ZSUM] = zs;
    }
    beta = (CT)b;
    zc = (CT)zcd;
  }
  const IO io(a, beta, zc);

  const int t = threadIdx.x, lane = t & 63;
  const int64_t cw = (int64_t)bx * (kThreads * 4) + (int64_t)(t >> 6) * 256;  // wave's first column
  const int64_t j0 = cw + 4 * lane;
  const bool active = j0 < a.ld;
  const int64_t r0 = (int64_t)by * rows_per_block;
  int64_t r1 = r0 + rows_per_block;
  if (r1 > a.Np) r1 = a.Np;
  const int64_t ld = a.ld;
  // rows the band reads: p from r0 - 1 to r1, the weights from r0 - 1 to
  // r1 - 1 (the loads one row ahead stop there instead of running past)
  const int64_t plim = r1 < a.Np ? r1 + 1 : a.Np;
  const int64_t wlim = r1;

  // weights of row i (zero outside the image rows)
  auto weights = [&](int64_t i, V4<CT>& ov, V4<CT>& oh) {
    ov = zero4<CT>();
    oh = zero4<CT>();
    if (active && i < wlim) {
      const V4<T> ovt = ld4_nt(a.Ov + i * ld + j0);
      const V4<T> oht = ld4_nt(a.Oh + i * ld + j0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ov.v[e] = (CT)ovt.v[e];
        oh.v[e] = (CT)oht.v[e];
      }
    }
  };
  // the wave's outside neighbours of row i: lane 0 gets p and the horizontal
  // weight left of the wave, lane 63 the p value right of it
  auto halo = [&](int64_t i, CT& hp, CT& hoh) {
    hp = (CT)0;
    hoh = (CT)0;
    if (i < wlim && cw < ld) {
      if (lane == 0 && cw > 0) {
        hp = io.p1(i, cw - 1);
        hoh = (CT)a.Oh[i * ld + cw - 1];
      } else if (lane == 63 && active) {
        hp = io.p1(i, cw + 256);
      }
    }
  };
  auto prow = [&](int64_t i) { return active && i < plim ? io.p4(i, j0) : zero4<CT>(); };

  V4<CT> pu = prow(r0 - 1), pc = prow(r0), pd = prow(r0 + 1), ovu = zero4<CT>();
  if (active && r0 > 0) {
    const V4<T> o = ld4_nt(a.Ov + (r0 - 1) * ld + j0);
#pragma unroll
    for (int e = 0; e < 4; ++e) ovu.v[e] = (CT)o.v[e];
  }
  V4<CT> ov, oh;
  weights(r0, ov, oh);
  CT hp, hoh;
  halo(r0, hp, hoh);

  double acc0 = 0.0, acc1 = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    // loads for the next rows, in flight while row i is computed
    const V4<CT> pn = prow(i + 2);
    V4<CT> ovn, ohn;
    weights(i + 1, ovn, ohn);
    CT hpn, hohn;
    halo(i + 1, hpn, hohn);

    CT pl = __shfl_up(pc.v[3], 1, 64);
    CT pr = __shfl_down(pc.v[0], 1, 64);
    CT ohl = __shfl_up(oh.v[3], 1, 64);
    if (lane == 0) {
      pl = hp;
      ohl = hoh;
    }
    if (lane == 63) pr = hp;
    if (active) {
      V4<CT> q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const CT right = e < 3 ? pc.v[e + 1] : pr;
        const CT left = e > 0 ? pc.v[e - 1] : pl;
        const CT wl = e > 0 ? oh.v[e - 1] : ohl;
        q.v[e] = ov.v[e] * (pc.v[e] - pd.v[e]) + ovu.v[e] * (pc.v[e] - pu.v[e]) +
                 oh.v[e] * (pc.v[e] - right) + wl * (pc.v[e] - left);
      }
      const int64_t o = i * ld + j0;
      if constexpr (MODE == ST_RESID) {
        const V4<T> bt = ld4_nt(a.b + o);
        V4<T> rt;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          rt.v[e] = (T)((double)bt.v[e] - q.v[e]);
          acc0 += (double)rt.v[e] * (double)rt.v[e];
          acc1 += (double)rt.v[e];
        }
        st4_nt(a.r + o, rt);
      } else {
        V4<T> qt;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          qt.v[e] = (T)q.v[e];
          acc0 += (double)pc.v[e] * (double)qt.v[e];
          if (MODE == ST_APPLY && a.want_qq) acc1 += (double)qt.v[e] * (double)qt.v[e];
        }
        st4_nt(a.q + o, qt);
        if constexpr (MODE == ST_FUSED) {
          V4<T> pt;
#pragma unroll
          for (int e = 0; e < 4; ++e) pt.v[e] = (T)pc.v[e];
          st4_nt(a.p_out + o, pt);
        }
      }
    }
    pu = pc;
    pc = pd;
    pd = pn;
    ovu = ov;
    ov = ovn;
    oh = ohn;
    hp = hpn;
    hoh = hohn;
  }

  if constexpr (MODE == ST_RESID) {
    double v[2] = {acc0, acc1};
    const int slots[2] = {PR_RR, PR_RSUM};
    write_partials<2>(a.st, slots, v, lb);
    // a larger partial count read by the consumers: the rest is zero
    if (threadIdx.x == 0 && a.nparts_out > 0) {
      const int nb = (int)(gridDim.x * gridDim.y);
      for (int k = lb + nb; k < a.nparts_out; k += nb) {
        part_row(a.st, PR_RR)[k] = 0.0;
        part_row(a.st, PR_RSUM)[k] = 0.0;
      }
    }
  } else if (MODE == ST_APPLY && a.want_qq) {
    double v[2] = {acc0, acc1};
    const int slots[2] = {PR_PQ, PR_AUX};
    write_partials<2>(a.st, slots, v, lb);
  } else {
    double v[1] = {acc0};
    const int slots[1] = {PR_PQ};
    write_partials<1>(a.st, slots, v, lb);
  }
}

template <class T, int MODE>
__global__ __launch_bounds__(kThreads) void stencil_kernel(StencilArgs<T> a, int rows_per_block) {
  stencil_body<T, MODE>(a, (int)blockIdx.x, (int)blockIdx.y, rows_per_block,
                        (int)(blockIdx.x + gridDim.x * blockIdx.y));
}

// Grouped launch over the tiles of a batch: block -> tile by binary search
// over the per-tile block prefix, then the tile's own arguments.
template <class T, int MODE>
__global__ __launch_bounds__(kThreads) void stencil_batched_kernel(const BatchTile<T>* tiles,
                                                                   const int32_t* start, int ntiles,
                                                                   int iter, int flexible,
                                                                   int check_done) {
  const int t = find_tile(start, ntiles, (int)blockIdx.x);
  const BatchTile<T>& bt = tiles[t];
  const int lb = (int)blockIdx.x - start[t];
  StencilArgs<T> a = batch_stencil_args<T>(bt, MODE, iter, flexible, check_done);
  stencil_body<T, MODE>(a, lb % bt.st_gx, lb / bt.st_gx, bt.st_rows, lb);
}

// Enough blocks to fill 256 CUs several times over, within the partials
// table; force_rows > 0 (a tuned band height) replaces the rule when its
// grid fits the table.
dim3 stencil_grid(int64_t Np, int64_t ld, int* rows_out, int force_rows) {
  const int64_t bx = (ld + 4 * kThreads - 1) / (4 * kThreads);
  int64_t rows = 64;
  while (rows > 4 && bx * ((Np + rows - 1) / rows) < 1024) rows /= 2;
  while (bx * ((Np + rows - 1) / rows) > kMaxPartials) rows *= 2;
  if (force_rows > 0 && bx * ((Np + force_rows - 1) / force_rows) <= kMaxPartials)
    rows = force_rows;
  *rows_out = (int)rows;
  return dim3((unsigned)bx, (unsigned)((Np + rows - 1) / rows));
}

template <class T>
int launch_stencil(int mode, const StencilArgs<T>& a, hipStream_t s) {
  int rows = 0;
  const dim3 grid = stencil_grid(a.Np, a.ld, &rows, a.rows);
  switch (mode) {
    case ST_FUSED:
      hipLaunchKernelGGL((stencil_kernel<T, ST_FUSED>), grid, dim3(kThreads), 0, s, a, rows);
      break;
    case ST_APPLY:
      hipLaunchKernelGGL((stencil_kernel<T, ST_APPLY>), grid, dim3(kThreads), 0, s, a, rows);
      break;
    default:
      hipLaunchKernelGGL((stencil_kernel<T, ST_RESID>), grid, dim3(kThreads), 0, s, a, rows);
      break;
  }
  return (int)(grid.x * grid.y);
}

template int launch_stencil<float>(int, const StencilArgs<float>&, hipStream_t);
template int launch_stencil<double>(int, const StencilArgs<double>&, hipStream_t);

template <class T>
void launch_stencil_batched(int mode, const BatchTile<T>* tiles, const int32_t* start, int ntiles,
                            int total_blocks, int iter, int flexible, int check_done,
                            hipStream_t s) {
  const dim3 grid((unsigned)total_blocks);
  switch (mode) {
    case ST_FUSED:
      hipLaunchKernelGGL((stencil_batched_kernel<T, ST_FUSED>), grid, dim3(kThreads), 0, s, tiles,
                         start, ntiles, iter, flexible, check_done);
      break;
    default:
      hipLaunchKernelGGL((stencil_batched_kernel<T, ST_RESID>), grid, dim3(kThreads), 0, s, tiles,
                         start, ntiles, iter, flexible, check_done);
      break;
  }
}

template void launch_stencil_batched<float>(int, const BatchTile<float>*, const int32_t*, int, int,
                                            int, int, int, hipStream_t);

}  // namespace irlsu
