// Packing and the structured matvec y = (S + sum u v^T) x and its transpose.
//
// Section 5.2 computes the block rank-one part in two phases: first one
// coefficient v . x_J per rank-one pair, then coefficient * u accumulated
// into the block row, on top of the CSR product of the sparse part.  Here one
// wavefront owns one block row (cell) and does both parts: phase 1 forms the
// coefficients of all pairs of the row with wave reductions, phase 2 streams
// the sparse rows and the u vectors once and writes y once.  The transpose
// gathers from the neighbours' records (block (nb, opposite d) multiplies x_nb
// into row c), so no atomics are needed and results are run-to-run
// deterministic.
//
// Pair counts: a diagonal block has g.rd pairs, a neighbour block g.ro.  The
// kernels are compiled for maxima RDM / ROM: <1, 1> is the one-pair-per-block
// layout (counts fixed at compile time), <9, 2> and <9, 6> take any rd <= 9
// and ro <= 2 or ro <= 6 with the counts as wave-uniform guards.
#include <type_traits>

#include "k_matvec_impl.hpp"

namespace r1s {

// ----------------------------------------------------------------- pack ----
// Block direction of pair slot q (slots ordered S, W, C, E, N).
__device__ inline int dir_of_slot(const Mesh& g, int q) {
  return q < g.ro ? D_S : q < 2 * g.ro ? D_W : q < 2 * g.ro + g.rd ? D_C
         : q < 3 * g.ro + g.rd ? D_E : D_N;
}

template <typename TV>
__global__ __launch_bounds__(256) void k_pack(Mesh g, PackIn in, TV* __restrict__ rec) {
  const long long RS = (long long)g.F * g.mp;
  const long long total = (long long)g.N * RS;
  const int L = g.L, m = g.m, P = g.P;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / RS);
    const int rem = (int)(idx - (long long)c * RS);
    const int f = rem / g.mp, k = rem - f * g.mp;
    double val = 0.0;
    if (k < m) {
      int nb[5];
      const int iy = c / g.nx, ix = c - iy * g.nx;
      nb[D_S] = iy > 0; nb[D_W] = ix > 0; nb[D_C] = 1;
      nb[D_E] = ix < g.nx - 1; nb[D_N] = iy < g.ny - 1;
      if (g.pat && (f == F_DIAG || f == F_LO || f == F_HI || (f >= g.fb && f < g.fu))) {
        // general pattern: diagonal, ELL and dense-index rows from the
        // entry table (F_LO / F_HI unused, zero)
        if (f == F_DIAG || f >= g.fb) {
          const int e = g.ppack[(f == F_DIAG ? 0 : f - g.fb + 1) * g.mp + k];
          if (e >= 0) val = in.s_cc[(long long)c * g.pnnz + e];
        }
      } else if (f == F_DIAG) {
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
      } else if (f < F_BAND) {
        const int slot = f - F_NBR;
        const int d = slot < 2 ? slot : slot + 1;
        if (nb[d]) val = in.s_nbr[((long long)c * 4 + slot) * m + k];
      } else if (f < g.fa) {
        // band row: lower j = 2..band, then upper; level rows only, entries
        // outside the block stay zero
        const int t = f - g.fb, nbd = g.band - 1;
        const int j = (t < nbd ? t : t - nbd) + 2;
        const bool ok = k < L && (t < nbd ? k >= j : k + j < L);
        if (ok) val = in.s_band[((long long)c * 2 * nbd + t) * L + k];
      } else if (f < g.fu) {
        // 0..2 level->flow, 3..5 flow->level; arrow = 2: 6 atom column, 7
        // atom row (inputs [N][4][L], slot 3; index a = L - 1 is not an entry)
        const int t = f - g.fa, ns = arrow_slots(g);
        const int slot = t < 6 ? t % 3 : 3;
        const bool lev_flow = t < 3 || t == 6;
        if (k < (t < 6 ? L : L - 1))
          val = (lev_flow ? in.s_lev_flow : in.s_flow_lev)[((long long)c * ns + slot) * L + k];
      } else if (f < g.fu + P) {
        const int q = f - g.fu;
        if (nb[dir_of_slot(g, q)]) val = in.u[((long long)c * P + q) * m + k];
      } else {
        const int q = f - g.fu - P;
        if (nb[dir_of_slot(g, q)]) val = in.v[((long long)c * P + q) * m + k];
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

// ------------------------------------------------------------ launchers ----
static inline int grid_for(long long work, int per_block, int cap = 1 << 20) {
  long long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_pack(const Mesh& g, const PackIn& in, double* rec64, float* rec32,
                       hipStream_t s) {
  const long long total = (long long)g.N * g.F * g.mp;
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

bool ranks_supported(int rd, int ro) {
  return rd >= 1 && rd <= RANK_DIAG_MAX && ro >= 0 && ro <= RANK_OFF_MAX;
}

// Right-hand sides per launch: 8 / 4 / 2 / 1 with one pair per block (4 / 2 / 1
// in the workgroup form), 2 / 1 with several (their coefficient registers
// grow with the pair count).
template <typename TV, bool TRANS, bool RESID>
static hipError_t launch_mv_t(const Mesh& g, const TV* rec, const double* x, const double* b,
                              double* y, int nrhs, hipStream_t s) {
  if (!ranks_supported(g.rd, g.ro) || g.band > BAND_MAX) return hipErrorInvalidValue;
  if (g.pat) {
    const int kind = (TRANS ? 1 : 0) | (RESID ? 2 : 0) | (std::is_same<TV, float>::value ? 4 : 0);
    return launch_mv_pattern(g, rec, kind, x, b, y, nrhs, s);
  }
  if (!wide_pattern(g) && g.rd == 1 && g.ro == 1) {
#ifndef R1S_NO_PACKED
    if (nrhs == 1 && packed_ok(g))
      return launch_matvec_packed(g, rec, std::is_same<TV, float>::value, TRANS, RESID, x, b, y, 0,
                                  s);
#endif
    return launch_mv_r<TV, TRANS, RESID, 1, 1, false>(g, rec, x, b, y, nrhs, s);
  }
  // several pairs per block or the wide diagonal block: the general
  // instantiations, compiled in files of their own
  const int kind = (TRANS ? 1 : 0) | (RESID ? 2 : 0) | (std::is_same<TV, float>::value ? 4 : 0);
  return g.ro <= RANK_OFF_SMALL ? launch_mv_general_r2(g, rec, kind, x, b, y, nrhs, s)
                                : launch_mv_general_r6(g, rec, kind, x, b, y, nrhs, s);
}

hipError_t launch_matvec(const Mesh& g, const void* rec, bool f32, bool trans, const double* x,
                         double* y, int nrhs, hipStream_t s) {
  if (g.graph) return launch_matvec_graph(g, rec, f32, trans, x, nullptr, y, nrhs, false, s);
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
  if (g.graph) return launch_matvec_graph(g, rec, false, trans, x, b, r, nrhs, true, s);
  return trans ? launch_mv_t<double, true, true>(g, rec, x, b, r, nrhs, s)
               : launch_mv_t<double, false, true>(g, rec, x, b, r, nrhs, s);
}

}  // namespace r1s
