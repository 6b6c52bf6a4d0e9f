// The matvec and the SMW block-Jacobi apply in one pass: z = M (J x), with y =
// J x written on the way (section 5.2 for the product, section 6 for the
// block-Jacobi step through the Woodbury identity; the operator M J is the
// one of the left-preconditioned system).
//
// The apply of cell c reads only y_c, and y_c is what the wave that owns
// cell c has just formed in its registers.  One wave per cell therefore
// computes y_c exactly as the single-chunk forward matvec does, stores it,
// and goes straight on to the local SMW solve exactly as the apply kernel
// does, so y is never read back from memory and the pair costs one launch.
// Single chunk (m <= 64), tridiagonal level band without level/flow
// coupling, one right-hand side per launch.
#include <type_traits>

#include "k_matvec_impl.hpp"

namespace r1s {

// EARLY: the factor rows of M are loaded together with the matrix rows (one
// memory round trip per wave); otherwise after the product, which keeps the
// register count down when the cell has many pairs.
template <typename TV, int RDM, int ROM, bool EARLY>
__global__ __launch_bounds__(64 * WPB) void k_matvec_prec(Mesh g_, const TV* __restrict__ rec,
                                                          const TV* __restrict__ fac,
                                                          const TV* __restrict__ invC,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ y,
                                                          double* __restrict__ z) {
  constexpr bool EXACT = RDM == 1 && ROM == 1;
  constexpr int RM = RDM > ROM ? RDM : ROM;
  const Mesh g = kmesh<EXACT>(g_);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c = __builtin_amdgcn_readfirstlane(tile * WPB + (int)(threadIdx.x >> 6));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, L = g.L;
  const long long mp = g.mp;
  const int kk = lane < m ? lane : m - 1;
  int nb[5], nbc[5], cnt[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
    cnt[d] = pair_count(g, d);
  }
  CellRows<TV, false> R;
  R.init(g, rec, c, nbc);

  // matrix rows and x blocks (missing neighbours read the cell's own rows and
  // are masked out of the sums)
  TV pv[5][RM], uv[5][RM], xv[5], nv[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
#pragma unroll
    for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
      pv[d][p] = p < cnt[d] ? ld_stream(R.base[d] + (R.coef0[d] + p) * mp + kk) : TV(0);
    xv[d] = (TV)x[(long long)nbc[d] * m + kk];
  }
  int pa, pb;
  if (kk < L) {
    pa = kk >= 1 ? kk - 1 : kk;
    pb = kk <= L - 2 ? kk + 1 : kk;
  } else {
    const int i = kk - L;
    pa = L + (i + 2) % 3;
    pb = L + (i + 1) % 3;
  }
  const TV dg = ld_stream(R.rc + F_DIAG * mp + kk);
  const TV ca = ld_stream(R.rc + F_LO * mp + kk);
  const TV cb = ld_stream(R.rc + F_HI * mp + kk);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C) nv[d] = ld_stream(R.base[d] + R.nbr[d] * mp + kk);
#pragma unroll
    for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
      uv[d][p] = p < cnt[d] ? ld_stream(R.base[d] + (R.out0[d] + p) * mp + kk) : TV(0);
  }

  // factor rows of the cell's diagonal block: bidiagonal sweeps (A, DI, B),
  // Woodbury W and V rows, C^{-1}
  const int rd = RDM == 1 ? 1 : g.rd;
  const TV* fc = fac + (long long)c * smw_rows(g) * mp;
  TV A[1], DI[1], B[1], W[RDM], V[RDM];
  CapInv<TV, RDM> IC;
  auto load_factors = [&]() {
    A[0] = ld_stream(fc + P_A * mp + kk);
    DI[0] = ld_stream(fc + P_DINV * mp + kk);
    B[0] = ld_stream(fc + P_B * mp + kk);
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      W[i] = i < rd ? ld_stream(fc + (P_W + i) * mp + kk) : TV(0);
      V[i] = i < rd ? ld_stream(fc + (P_W + rd + i) * mp + kk) : TV(0);
    }
    IC.load(invC, c, rd, lane);
  };
  if constexpr (EARLY) load_factors();
  __builtin_amdgcn_sched_barrier(0);

  // y_c = (S + sum u v^T) x restricted to block row c (the coefficient sums
  // as the matvec kernel forms them, so that y is bitwise its result)
  TV acc[5][RM];
  constexpr int NSUM = RDM + 4 * ROM;
#pragma unroll
  for (int g0 = 0; g0 < NSUM; g0 += 4) {
    TV s4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      s4[e] = TV(0);
      if (g0 + e < NSUM) {
        int d, p;
        pair_index<RDM, ROM>(g0 + e, d, p);
        if (lane < m) s4[e] += pv[d][p] * xv[d];
      }
    }
    wave_sums_u(s4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (g0 + e < NSUM) {
        int d, p;
        pair_index<RDM, ROM>(g0 + e, d, p);
        acc[d][p] = ex[d] ? s4[e] : TV(0);
      }
    }
  }
  const TV xa = __shfl(xv[D_C], pa, WAVE), xb = __shfl(xv[D_C], pb, WAVE);
  TV t = dg * xv[D_C] + ca * xa + cb * xb;
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C && ex[d]) t += nv[d] * xv[d];
#pragma unroll
    for (int p = 0; p < (d == D_C ? RDM : ROM); ++p) t += uv[d][p] * acc[d][p];
  }
  const double yv = (double)t;
  st_out(y + (long long)c * m + kk, yv);  // lanes past m repeat lane m-1's value

  // z_c = x0 - W C^{-1} (V^T x0), x0 = A0^{-1} y_c
  if constexpr (!EARLY) load_factors();
  const TV r[1] = {(TV)yv};
  TV X0[1];
  smw_sweeps<TV, 1, false>(L, m, A, DI, B, r, lane_value<TV, 1>(r, L),
                           lane_value<TV, 1>(r, L + 1), lane_value<TV, 1>(r, L + 2), X0);
  TV s[RDM], zc[RDM];
#pragma unroll
  for (int i = 0; i < RDM; ++i) {
    TV tv = TV(0);
    tv += V[i] * X0[0];
    s[i] = i < rd ? wave_sum_u(tv) : TV(0);
  }
  IC.template apply<false>(s, zc, rd);
  TV o = X0[0];
#pragma unroll
  for (int i = 0; i < RDM; ++i) o -= zc[i] * W[i];
  if (lane < m) st_out(z + (long long)c * m + lane, (double)o);
}

// Where the single kernel is used: the layouts it covers, and among them
// those where it measured faster than the two kernels (256 x 128, L = 61:
// one pair per block 69.4 against 72.1 us in float64, 37.5 against 43.3 us
// with float32 values; with 9 / 2 or 2 / 6 pairs the float64 form holds
// 120-190 registers, runs at 2-4 waves per SIMD and was 2-7% slower).
bool matvec_prec_fused(const Mesh& g, bool f32) {
  const bool covered = !g.graph && g.m <= WAVE && !wide_pattern(g) && g.rd >= 1 &&
                       g.rd <= RANK_DIAG_MAX && g.ro >= 0 && g.ro <= RANK_OFF_MAX;
  return covered && (f32 || (g.rd == 1 && g.ro == 1));
}

template <typename TV, int RDM, int ROM, bool EARLY>
static hipError_t launch_mp(const Mesh& g, const TV* rec, const TV* fac, const TV* invC,
                            const double* x, double* y, double* z, hipStream_t s) {
  const int grid = (g.N + WPB - 1) / WPB;
  hipLaunchKernelGGL((k_matvec_prec<TV, RDM, ROM, EARLY>), dim3(grid), dim3(64 * WPB), 0, s, g,
                     rec, fac, invC, x, y, z);
  return hipGetLastError();
}

template <typename TV>
static hipError_t launch_mp_t(const Mesh& g, const TV* rec, const TV* fac, const TV* invC,
                              const double* x, double* y, double* z, hipStream_t s) {
  if (g.rd == 1 && g.ro == 1)
    return launch_mp<TV, 1, 1, true>(g, rec, fac, invC, x, y, z, s);
  if constexpr (std::is_same<TV, float>::value) {  // several pairs: float32 only
    if (g.ro <= RANK_OFF_SMALL)
      return launch_mp<TV, RANK_DIAG_MAX, RANK_OFF_SMALL, false>(g, rec, fac, invC, x, y, z, s);
    return launch_mp<TV, RANK_DIAG_MAX, RANK_OFF_MAX, false>(g, rec, fac, invC, x, y, z, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_matvec_prec(const Mesh& g, const void* rec, const void* fac, const void* invC,
                              bool f32, const double* x, double* y, double* z, hipStream_t s) {
  if (!matvec_prec_fused(g, f32)) return hipErrorInvalidValue;
  if (f32)
    return launch_mp_t<float>(g, (const float*)rec, (const float*)fac, (const float*)invC, x, y,
                              z, s);
  return launch_mp_t<double>(g, (const double*)rec, (const double*)fac, (const double*)invC, x, y,
                             z, s);
}

}  // namespace r1s
