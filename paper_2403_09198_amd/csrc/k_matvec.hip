// Packing and the structured matvec y = (S + sum u v^T) x and its transpose.
//
// Section 5.2 computes the block rank-one part in two phases: first one
// coefficient v . x_J per rank-one pair, then coefficient * u accumulated
// into the block row, on top of the CSR product of the sparse part.  Here one
// wavefront owns one block row (cell) and does both parts: phase 1 forms the
// five pair coefficients with wave reductions, phase 2 streams the sparse
// rows and the u vectors once and writes y once.  The transpose gathers from
// the neighbours' records (block (nb, opposite d) multiplies x_nb into row c),
// so no atomics are needed and results are run-to-run deterministic.
#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

// ----------------------------------------------------------------- pack ----
template <typename TV>
__global__ __launch_bounds__(256) void k_pack(Mesh g, PackIn in, TV* __restrict__ rec) {
  const long long total = (long long)g.N * F_REC * g.mp;
  const int L = g.L, m = g.m;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / (F_REC * g.mp));
    const int rem = (int)(idx - (long long)c * F_REC * g.mp);
    const int f = rem / g.mp, k = rem - f * g.mp;
    double val = 0.0;
    if (k < m) {
      int nb[5];
      const int iy = c / g.nx, ix = c - iy * g.nx;
      nb[D_S] = iy > 0; nb[D_W] = ix > 0; nb[D_C] = 1;
      nb[D_E] = ix < g.nx - 1; nb[D_N] = iy < g.ny - 1;
      if (f == F_DIAG) {
        val = in.s_diag[(long long)c * m + k];
      } else if (f == F_LO || f == F_HI) {
        if (k < L) {
          if (f == F_LO && k >= 1) val = in.s_sub[(long long)c * (L - 1) + k - 1];
          if (f == F_HI && k <= L - 2) val = in.s_sup[(long long)c * (L - 1) + k];
        } else {
          const int i = k - L;
          const int j = f == F_LO ? (i + 2) % 3 : (i + 1) % 3;
          val = in.s_flow[(long long)c * 6 + i * 2 + (j > i ? j - 1 : j)];
        }
      } else if (f < F_U) {
        const int slot = f - F_NBR;
        const int d = slot < 2 ? slot : slot + 1;
        if (nb[d]) val = in.s_nbr[((long long)c * 4 + slot) * m + k];
      } else if (f < F_V) {
        const int d = f - F_U;
        if (nb[d]) val = in.u[((long long)c * 5 + d) * m + k];
      } else {
        const int d = f - F_V;
        if (nb[d]) val = in.v[((long long)c * 5 + d) * m + k];
      }
    }
    rec[idx] = (TV)val;
  }
}

template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_cast(const TI* __restrict__ src, TO* __restrict__ dst,
                                              long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (TO)src[i];
}

// --------------------------------------------------------------- matvec ----
// TV: value / accumulation type.  NCH = ceil(m / 64) chunks of 64 unknowns,
// NR right-hand sides per launch starting at rhs r0.  RESID: write b - J x.
//
// Every load of a wave is independent of the reductions, so all of them are
// issued before the first wait: missing neighbours (mesh boundary) read the
// cell's own, valid addresses and are masked out of the sums instead of
// being skipped by a branch.  Lanes past m read element m-1 and are masked.
template <typename TV, int NCH, int NR, bool TRANS, bool RESID>
__global__ __launch_bounds__(64 * WPB) void k_matvec(Mesh g, const TV* __restrict__ rec,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b,
                                                double* __restrict__ y, int r0) {
  constexpr bool PRELOAD = NCH == 1;  // hold the sparse rows across the reduction
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c = __builtin_amdgcn_readfirstlane(tile * WPB + (int)(threadIdx.x >> 6));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, mp = g.mp, L = g.L;
  const long long RS = (long long)F_REC * mp;
  int nb[5], nbc[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
  }
  const TV* rc = rec + (long long)c * RS;
  // coefficient row of phase 1, output row of phase 2, neighbour diagonal
  const TV* prow[5];
  const TV* urow[5];
  const TV* nrow[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (!TRANS) {
      prow[d] = rc + (long long)(F_V + d) * mp;
      urow[d] = rc + (long long)(F_U + d) * mp;
      nrow[d] = rc + (long long)(F_NBR + nbr_slot(d == D_C ? 0 : d)) * mp;
    } else {
      const TV* rn = rec + (long long)nbc[d] * RS;
      prow[d] = rn + (long long)(F_U + opposite(d)) * mp;
      urow[d] = rn + (long long)(F_V + opposite(d)) * mp;
      nrow[d] = rn + (long long)(F_NBR + nbr_slot(d == D_C ? 0 : opposite(d))) * mp;
    }
  }
  const double* xr = x + (long long)r0 * g.n;

  TV pv[5][NCH], xv[NR][5][NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      pv[d][ch] = ld_stream(prow[d] + kk);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        xv[r][d][ch] = (TV)xr[(long long)r * g.n + (long long)nbc[d] * m + kk];
    }
  }

  // sparse part of the row: diagonal, level band / flow corner partners,
  // neighbour diagonals, and the u rows
  TV dg[NCH], ca[NCH], cb[NCH], nv[5][NCH], uv[5][NCH], xa[NR][NCH], xb[NR][NCH];
  auto load_sparse = [&](int ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
    int pa, pb;
    bool va, vb;
    if (kk < L) {
      va = kk >= 1; pa = va ? kk - 1 : kk;
      vb = kk <= L - 2; pb = vb ? kk + 1 : kk;
    } else {
      const int i = kk - L;
      pa = L + (i + 2) % 3; va = true;
      pb = L + (i + 1) % 3; vb = true;
    }
    dg[ch] = ld_stream(rc + (long long)F_DIAG * mp + kk);
    if (!TRANS) {  // row k of S_cc: lo at column pa, hi at column pb
      ca[ch] = ld_stream(rc + (long long)F_LO * mp + kk);
      cb[ch] = ld_stream(rc + (long long)F_HI * mp + kk);
    } else {       // column k of S_cc: hi of row pa, lo of row pb
      const TV ta = rc[(long long)F_HI * mp + pa];
      const TV tb = rc[(long long)F_LO * mp + pb];
      ca[ch] = va ? ta : TV(0);
      cb[ch] = vb ? tb : TV(0);
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (d != D_C) nv[d][ch] = ld_stream(nrow[d] + kk);
      uv[d][ch] = ld_stream(urow[d] + kk);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double* xv_c = xr + (long long)r * g.n + (long long)c * m;
      xa[r][ch] = (TV)xv_c[pa];
      xb[r][ch] = (TV)xv_c[pb];
    }
  };
  if (PRELOAD) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) load_sparse(ch);
    // keep these loads in flight during the reductions (one memory round
    // trip per wave instead of two)
    __builtin_amdgcn_sched_barrier(0);
  }

  // pair coefficients: forward v_{c,d} . x_nb, transpose u_{nb,opp d} . x_nb
  TV acc[NR][5];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      TV s = TV(0);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (ch * WAVE + lane < m) s += pv[d][ch] * xv[r][d][ch];
      s = wave_sum_u(s);
      acc[r][d] = ex[d] ? s : TV(0);
    }

  // Lanes past m computed exactly what lane m-1 computes (all their indices
  // are clamped), so every lane stores to its clamped index: duplicate lanes
  // write identical values and no branch is needed around the stores.
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    if (!PRELOAD) load_sparse(ch);
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      TV t = dg[ch] * xv[r][D_C][ch] + ca[ch] * xa[r][ch] + cb[ch] * xb[r][ch];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        if (d != D_C && ex[d]) t += nv[d][ch] * xv[r][d][ch];
        t += uv[d][ch] * acc[r][d];
      }
      const long long o = (long long)(r0 + r) * g.n + (long long)c * m + kk;
      y[o] = RESID ? b[o] - (double)t : (double)t;
    }
  }
}

// Workgroup-per-cell form for m > 64: wave w of the workgroup owns unknowns
// 64w .. 64w+63 of one cell, issues all of its loads at once (like the
// single-chunk kernel), and the five pair coefficients are summed over the
// waves through LDS in a fixed order.
template <typename TV, int NCH, int NR, bool TRANS, bool RESID>
__global__ __launch_bounds__(64 * NCH) void k_matvec_wg(Mesh g, const TV* __restrict__ rec,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ y, int r0) {
  __shared__ TV part[NR][5][NCH];
  const int c = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const int m = g.m, mp = g.mp, L = g.L;
  const long long RS = (long long)F_REC * mp;
  int nb[5], nbc[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
  }
  const TV* rc = rec + (long long)c * RS;
  const TV* prow[5];
  const TV* urow[5];
  const TV* nrow[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (!TRANS) {
      prow[d] = rc + (long long)(F_V + d) * mp;
      urow[d] = rc + (long long)(F_U + d) * mp;
      nrow[d] = rc + (long long)(F_NBR + nbr_slot(d == D_C ? 0 : d)) * mp;
    } else {
      const TV* rn = rec + (long long)nbc[d] * RS;
      prow[d] = rn + (long long)(F_U + opposite(d)) * mp;
      urow[d] = rn + (long long)(F_V + opposite(d)) * mp;
      nrow[d] = rn + (long long)(F_NBR + nbr_slot(d == D_C ? 0 : opposite(d))) * mp;
    }
  }
  const double* xr = x + (long long)r0 * g.n;
  const int k = wv * WAVE + lane;
  const int kk = k < m ? k : m - 1;

  TV pv[5], xv[NR][5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    pv[d] = ld_stream(prow[d] + kk);
#pragma unroll
    for (int r = 0; r < NR; ++r) xv[r][d] = (TV)xr[(long long)r * g.n + (long long)nbc[d] * m + kk];
  }
  int pa, pb;
  bool va, vb;
  if (kk < L) {
    va = kk >= 1; pa = va ? kk - 1 : kk;
    vb = kk <= L - 2; pb = vb ? kk + 1 : kk;
  } else {
    const int i = kk - L;
    pa = L + (i + 2) % 3; va = true;
    pb = L + (i + 1) % 3; vb = true;
  }
  const TV dg = ld_stream(rc + (long long)F_DIAG * mp + kk);
  TV ca, cb;
  if (!TRANS) {
    ca = ld_stream(rc + (long long)F_LO * mp + kk);
    cb = ld_stream(rc + (long long)F_HI * mp + kk);
  } else {
    const TV ta = rc[(long long)F_HI * mp + pa];
    const TV tb = rc[(long long)F_LO * mp + pb];
    ca = va ? ta : TV(0);
    cb = vb ? tb : TV(0);
  }
  TV nv[5], uv[5], xa[NR], xb[NR];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C) nv[d] = ld_stream(nrow[d] + kk);
    uv[d] = ld_stream(urow[d] + kk);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double* xv_c = xr + (long long)r * g.n + (long long)c * m;
    xa[r] = (TV)xv_c[pa];
    xb[r] = (TV)xv_c[pb];
  }
  __builtin_amdgcn_sched_barrier(0);

#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      const TV s = wave_sum_u(k < m ? pv[d] * xv[r][d] : TV(0));
      if (lane == 0) part[r][d][wv] = s;
    }
  __syncthreads();
  TV acc[NR][5];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      TV s = part[r][d][0];
#pragma unroll
      for (int w = 1; w < NCH; ++w) s += part[r][d][w];
      acc[r][d] = ex[d] ? s : TV(0);
    }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    TV t = dg * xv[r][D_C] + ca * xa[r] + cb * xb[r];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (d != D_C && ex[d]) t += nv[d] * xv[r][d];
      t += uv[d] * acc[r][d];
    }
    const long long o = (long long)(r0 + r) * g.n + (long long)c * m + kk;
    y[o] = RESID ? b[o] - (double)t : (double)t;
  }
}

// ------------------------------------------------------------ launchers ----
static inline int grid_for(long long work, int per_block, int cap = 1 << 20) {
  long long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_pack(const Mesh& g, const PackIn& in, double* rec64, float* rec32,
                       hipStream_t s) {
  const long long total = (long long)g.N * F_REC * g.mp;
  hipLaunchKernelGGL(k_pack<double>, dim3(grid_for(total, 256, 65536)), dim3(256), 0, s, g, in,
                     rec64);
  if (rec32)
    hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(total, 256, 65536)), dim3(256), 0, s,
                       rec64, rec32, total);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* src, float* dst, long long count, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(count, 256, 65536)), dim3(256), 0, s,
                     src, dst, count);
  return hipGetLastError();
}

template <typename TV, int NCH, bool TRANS, bool RESID>
static void launch_mv_nch(const Mesh& g, const TV* rec, const double* x, const double* b,
                          double* y, int nrhs, hipStream_t s) {
#ifndef R1S_NO_WG_CELL
  if constexpr (NCH > 1) {
    int r0 = 0;
    while (r0 < nrhs) {
      const int rem = nrhs - r0;
      if (rem >= 4) {
        hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 4, TRANS, RESID>), dim3(g.N), dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
        r0 += 4;
      } else if (rem >= 2) {
        hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 2, TRANS, RESID>), dim3(g.N), dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
        r0 += 2;
      } else {
        hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 1, TRANS, RESID>), dim3(g.N), dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
        r0 += 1;
      }
    }
    return;
  }
#endif
  const int grid = (g.N + WPB - 1) / WPB;
  int r0 = 0;
  while (r0 < nrhs) {
    const int rem = nrhs - r0;
    if constexpr (NCH <= 2) {
      if (rem >= 8) {
        hipLaunchKernelGGL((k_matvec<TV, NCH, 8, TRANS, RESID>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, x, b, y, r0);
        r0 += 8;
        continue;
      }
      if (rem >= 4) {
        hipLaunchKernelGGL((k_matvec<TV, NCH, 4, TRANS, RESID>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, x, b, y, r0);
        r0 += 4;
        continue;
      }
    }
    if (rem >= 2) {
      hipLaunchKernelGGL((k_matvec<TV, NCH, 2, TRANS, RESID>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, x, b, y, r0);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_matvec<TV, NCH, 1, TRANS, RESID>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, x, b, y, r0);
      r0 += 1;
    }
  }
}

template <typename TV, bool TRANS, bool RESID>
static hipError_t launch_mv_t(const Mesh& g, const TV* rec, const double* x, const double* b,
                              double* y, int nrhs, hipStream_t s) {
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: launch_mv_nch<TV, 1, TRANS, RESID>(g, rec, x, b, y, nrhs, s); break;
    case 2: launch_mv_nch<TV, 2, TRANS, RESID>(g, rec, x, b, y, nrhs, s); break;
    case 3: launch_mv_nch<TV, 3, TRANS, RESID>(g, rec, x, b, y, nrhs, s); break;
    case 4: launch_mv_nch<TV, 4, TRANS, RESID>(g, rec, x, b, y, nrhs, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_matvec(const Mesh& g, const void* rec, bool f32, bool trans, const double* x,
                         double* y, int nrhs, hipStream_t s) {
  if (f32) {
    const float* r = (const float*)rec;
    return trans ? launch_mv_t<float, true, false>(g, r, x, nullptr, y, nrhs, s)
                 : launch_mv_t<float, false, false>(g, r, x, nullptr, y, nrhs, s);
  }
  const double* r = (const double*)rec;
  return trans ? launch_mv_t<double, true, false>(g, r, x, nullptr, y, nrhs, s)
               : launch_mv_t<double, false, false>(g, r, x, nullptr, y, nrhs, s);
}

hipError_t launch_residual(const Mesh& g, const double* rec, bool trans, const double* b,
                           const double* x, double* r, int nrhs, hipStream_t s) {
  return trans ? launch_mv_t<double, true, true>(g, rec, x, b, r, nrhs, s)
               : launch_mv_t<double, false, true>(g, rec, x, b, r, nrhs, s);
}

}  // namespace r1s
