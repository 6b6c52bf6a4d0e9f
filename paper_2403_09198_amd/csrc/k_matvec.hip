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
// TV: value / accumulation type.  NR right-hand sides per launch, starting
// at rhs r0.  RESID: write b - J x instead of J x.
template <typename TV, int NR, bool TRANS, bool RESID>
__global__ __launch_bounds__(256) void k_matvec(Mesh g, const TV* __restrict__ rec,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b,
                                                double* __restrict__ y, int r0) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c = __builtin_amdgcn_readfirstlane(tile * 4 + (int)(threadIdx.x >> 6));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, mp = g.mp, L = g.L;
  const long long RS = (long long)F_REC * mp;
  int nb[5];
  neighbours(g, c, nb);
  const TV* rc = rec + (long long)c * RS;
  const double* xr = x + (long long)r0 * g.n;

  // Phase 1: one coefficient per block of the row (forward: v_{c,d} . x_nb;
  // transpose: u_{nb,opp d} . x_nb).
  TV acc[NR][5];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int d = 0; d < 5; ++d) acc[r][d] = TV(0);
  for (int k0 = 0; k0 < m; k0 += WAVE) {
    const int k = k0 + lane;
    if (k < m) {
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        if (nb[d] < 0) continue;
        const TV* src = TRANS ? rec + (long long)nb[d] * RS + (long long)(F_U + opposite(d)) * mp
                              : rc + (long long)(F_V + d) * mp;
        const TV vv = src[k];
#pragma unroll
        for (int r = 0; r < NR; ++r)
          acc[r][d] += vv * (TV)xr[(long long)r * g.n + (long long)nb[d] * m + k];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int d = 0; d < 5; ++d) acc[r][d] = wave_sum(acc[r][d]);

  // Phase 2: sparse part + rank-one accumulation, one pass over the row.
  for (int k0 = 0; k0 < m; k0 += WAVE) {
    const int k = k0 + lane;
    if (k >= m) continue;
    // partner columns of the diagonal block: level band k-1 / k+1, or the
    // two other flow unknowns
    int pa, pb;
    bool va, vb;
    if (k < L) {
      pa = k - 1; va = k >= 1;
      pb = k + 1; vb = k <= L - 2;
    } else {
      const int i = k - L;
      pa = L + (i + 2) % 3; va = true;
      pb = L + (i + 1) % 3; vb = true;
    }
    const TV dg = rc[(long long)F_DIAG * mp + k];
    TV ca, cb;
    if (!TRANS) {  // row k of S_cc: lo at column pa, hi at column pb
      ca = rc[(long long)F_LO * mp + k];
      cb = rc[(long long)F_HI * mp + k];
    } else {       // column k of S_cc: hi of row pa, lo of row pb
      ca = va ? rc[(long long)F_HI * mp + pa] : TV(0);
      cb = vb ? rc[(long long)F_LO * mp + pb] : TV(0);
    }
    if (!va) pa = k;
    if (!vb) pb = k;
    TV t[NR];
    const long long xc = (long long)c * m;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double* xv = xr + (long long)r * g.n + xc;
      t[r] = dg * (TV)xv[k] + ca * (TV)xv[pa] + cb * (TV)xv[pb];
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (nb[d] < 0) continue;
      if (d != D_C) {
        const TV cn = TRANS ? rec[(long long)nb[d] * RS + (long long)(F_NBR + nbr_slot(opposite(d))) * mp + k]
                            : rc[(long long)(F_NBR + nbr_slot(d)) * mp + k];
#pragma unroll
        for (int r = 0; r < NR; ++r)
          t[r] += cn * (TV)xr[(long long)r * g.n + (long long)nb[d] * m + k];
      }
      const TV uu = TRANS ? rec[(long long)nb[d] * RS + (long long)(F_V + opposite(d)) * mp + k]
                          : rc[(long long)(F_U + d) * mp + k];
#pragma unroll
      for (int r = 0; r < NR; ++r) t[r] += uu * acc[r][d];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const long long o = (long long)(r0 + r) * g.n + xc + k;
      y[o] = RESID ? b[o] - (double)t[r] : (double)t[r];
    }
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

template <typename TV, bool TRANS, bool RESID>
static hipError_t launch_mv_t(const Mesh& g, const TV* rec, const double* x, const double* b,
                              double* y, int nrhs, hipStream_t s) {
  const int grid = (g.N + 3) / 4;
  int r0 = 0;
  while (r0 < nrhs) {
    const int rem = nrhs - r0;
    if (rem >= 8) {
      hipLaunchKernelGGL((k_matvec<TV, 8, TRANS, RESID>), dim3(grid), dim3(256), 0, s, g, rec, x, b, y, r0);
      r0 += 8;
    } else if (rem >= 4) {
      hipLaunchKernelGGL((k_matvec<TV, 4, TRANS, RESID>), dim3(grid), dim3(256), 0, s, g, rec, x, b, y, r0);
      r0 += 4;
    } else if (rem >= 2) {
      hipLaunchKernelGGL((k_matvec<TV, 2, TRANS, RESID>), dim3(grid), dim3(256), 0, s, g, rec, x, b, y, r0);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_matvec<TV, 1, TRANS, RESID>), dim3(grid), dim3(256), 0, s, g, rec, x, b, y, r0);
      r0 += 1;
    }
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
