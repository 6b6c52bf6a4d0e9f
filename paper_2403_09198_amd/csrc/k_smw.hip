// Block-Jacobi preconditioner through the Sherman-Morrison-Woodbury identity.
//
// Section 6: the diagonal block of cell c is D_c = A0_c + U V^T (eq.
// R1_Block_Jacobian) with A0_c the sparse diagonal block of S and the rd
// columns of U, V the block's rank-one pairs.  With W = A0^{-1} U and the rd x
// rd capacitance C = I + V^T W (SMW-1, SMW-2), D_c^{-1} r = x0 - W C^{-1} V^T x0
// where x0 = A0^{-1} r.  The printed identity adds the correction; the correct
// Woodbury identity subtracts it, which is what is computed here.  With one
// pair C is the scalar 1 + v . w.
//
// A0_c is the tridiagonal level band T plus a dense 3 x 3 flow corner F,
// optionally with level/flow coupling (dense level rows x flow columns Ec
// and flow rows x level columns Er).  The band is factored once (LU without
// pivoting, the Thomas algorithm); each apply then runs the two bidiagonal
// sweeps as affine-map scans across the 64 lanes of one wavefront (a serial
// recurrence y_k = a_k y_{k-1} + b_k is a prefix composition of affine
// maps), carrying the last value from one 64-level chunk to the next.  The
// coupling is eliminated through the 3 x 3 Schur complement S3 = F - Er
// T^{-1} Ec, which takes the place of F^{-1} in the factor record.
//
// With the atom density coupled to every molecule level (arrow = 2, a dense
// column and row through the band), A0 keeps the three-slot pattern and the
// atom's column c and row r join the Woodbury terms as two more pairs,
// D_c = A0 + U V^T + c e_a^T + e_a r^T: the band sweeps stay affine scans and
// the capacitance grows from rd x rd to (rd + 2) x (rd + 2).
#include <math.h>

#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

__global__ void k_fill_int(int* p, int value, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

hipError_t launch_fill_int(int* p, int value, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- setup ----
// One wavefront per cell, NCH chunks of 64 unknowns, runs once per matrix.
//
// Band LU (Thomas algorithm, no pivoting): d_0 = a_0, d_k = a_k - e_k / d_{k-1}
// with e_k = sub_{k-1} sup_{k-1}.  The pivots are a continued fraction: with
// d_k = p_k / q_k, [p_k; q_k] = [[a_k, -e_k], [1, 0]] [p_{k-1}; q_{k-1}], so
// every chunk runs one inclusive scan of 2 x 2 matrix products (each factor
// scaled by 1 / max(|a_k|, |e_k|, 1), which leaves the ratio unchanged and
// keeps 64-factor products far from overflow) applied to the carried
// [d_{prev}; 1].  Then l_k = sub_{k-1} / d_{k-1}, and the factor rows:
//   forward  a = -l_k, dinv = 1/d_k, b = -sup_k / d_k, W_i = A0^{-1} u_i, v_i
//   transpose a = -sup_{k-1} / d_k, dinv, b = -l_{k+1}, A0^{-T} v_i, u_i
// Flow lanes L + i hold row i of the 3 x 3 corner inverse (transpose: of its
// transpose).  W uses the same affine-scan sweeps as the apply.
//
// C^{-1} by Gauss-Jordan elimination with partial pivoting on [C | I]: lane t
// holds column t of the augmented matrix (rows in registers), pivots are read
// with v_readlane, so every step is wave-uniform.  The transposed apply uses
// (C^{-1})^T, since I + U^T A0^{-T} V = C^T.
template <int NCH, int RDM>
__global__ __launch_bounds__(64 * WPB) void k_smw_setup(Mesh g, const double* __restrict__ rec,
                                                       double* __restrict__ facF,
                                                       double* __restrict__ facT,
                                                       double* __restrict__ invC, int* status) {
  const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + (threadIdx.x >> 6)));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int L = g.L, m = g.m, mp = g.mp;
  const int rd = RDM == 1 ? 1 : smw_pairs(g);  // Woodbury terms
  const int rdu = RDM == 1 ? 1 : g.rd;          // of them, the block's own pairs
  const int SR = smw_rows(g);
  const bool arw = g.arrow;  // wave-uniform
  const double* rc = rec + (long long)c * g.F * mp;
  const double* dg = rc + (long long)F_DIAG * mp;
  const double* lo = rc + (long long)F_LO * mp;
  const double* hi = rc + (long long)F_HI * mp;
  const double* uC = rc + (long long)(g.fu + pair_start(g, D_C)) * mp;         // pair i at + i mp
  const double* vC = rc + (long long)(g.fu + g.P + pair_start(g, D_C)) * mp;
  // pair j's u and v at element kk (kk < m): the block's pairs, then the
  // atom's column (u = column, v = e_a) and row (u = e_a, v = row)
  const int ia = L - 1;
  auto pair_u = [&](int j, int kk) -> double {
    if (j < rdu) return uC[j * mp + kk];
    if (j == rdu) return kk < ia ? rc[(long long)arrow_col_row(g, 3) * mp + kk] : 0.0;
    return kk == ia ? 1.0 : 0.0;
  };
  auto pair_v = [&](int j, int kk) -> double {
    if (j < rdu) return vC[j * mp + kk];
    if (j == rdu) return kk == ia ? 1.0 : 0.0;
    return kk < ia ? rc[(long long)arrow_row_row(g, 3) * mp + kk] : 0.0;
  };

  double AD[NCH], LO[NCH], HI[NCH], HM1[NCH], LP1[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
    AD[ch] = dg[kk];
    LO[ch] = lo[kk];
    HI[ch] = hi[kk];
    HM1[ch] = kk >= 1 ? hi[kk - 1] : 0.0;
    LP1[ch] = kk + 1 < m ? lo[kk + 1] : 0.0;
  }
  // 3 x 3 flow corner (wave-uniform values), inverse by cofactors
  double F[3][3], Fi[3][3];
  for (int i = 0; i < 3; ++i) {
    F[i][i] = dg[L + i];
    F[i][(i + 2) % 3] = lo[L + i];
    F[i][(i + 1) % 3] = hi[L + i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
      Fi[i][j] = F[r1][c1] * F[r2][c2] - F[r1][c2] * F[r2][c1];  // adjugate
    }
  const double det = F[0][0] * Fi[0][0] + F[0][1] * Fi[1][0] + F[0][2] * Fi[2][0];
  double rn = 1.0;
  for (int i = 0; i < 3; ++i) rn *= fabs(F[i][0]) + fabs(F[i][1]) + fabs(F[i][2]);
  // with coupling only the Schur complement must be regular (below)
  bool bad = !arw && !(fabs(det) > 1e-14 * rn);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Fi[i][j] = arw ? 0.0 : Fi[i][j] / det;

  // pivots d_k by the matrix-product scan, chunk by chunk
  double D[NCH], DP[NCH];  // d_k and d_{k-1}
  double dprev = 1.0, qprev = 0.0;  // [p_{-1}; q_{-1}] = [1; 0]
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const bool lev = k < L;
    const double e = k >= 1 ? LO[ch] * HM1[ch] : 0.0;
    const double sc = 1.0 / fmax(fmax(fabs(AD[ch]), fabs(e)), 1.0);
    double ma = lev ? AD[ch] * sc : 1.0, mb = lev ? -e * sc : 0.0;
    double mc = lev ? sc : 0.0, md = lev ? 0.0 : 1.0;
    if (ch * WAVE < L) {
      scan_mat2_up_dpp(ma, mb, mc, md);
      const double p = ma * dprev + mb * qprev;
      const double q = mc * dprev + md * qprev;
      D[ch] = p / q;
      // d_{k-1}: one lane up; lane 0 takes the previous chunk's last pivot
      const double up = __shfl_up(D[ch], 1, WAVE);
      DP[ch] = lane == 0 ? dprev / qprev : up;
      if (ch == 0 && lane == 0) DP[ch] = 1.0;
      dprev = readlane(D[ch], WAVE - 1);
      qprev = 1.0;
    } else {
      D[ch] = 1.0;
      DP[ch] = 1.0;
    }
  }
  // factor rows
  double FA[NCH], FDI[NCH], FB[NCH], TA[NCH], TDI[NCH], TB[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    if (k < L) {
      const double l = k >= 1 ? LO[ch] / DP[ch] : 0.0;
      const double t = k >= 1 ? l * HM1[ch] : 0.0;
      if (!(fabs(D[ch]) > 1e-14 * (fabs(AD[ch]) + fabs(t)))) bad = true;
      const double di = 1.0 / D[ch];
      FA[ch] = -l;
      FDI[ch] = di;
      FB[ch] = k <= L - 2 ? -HI[ch] * di : 0.0;
      TA[ch] = k >= 1 ? -HM1[ch] * di : 0.0;
      TDI[ch] = di;
      TB[ch] = k <= L - 2 ? -LP1[ch] * di : 0.0;
    } else {
      const int i = k - L < 3 ? k - L : 0;
      FA[ch] = Fi[i][0];
      FDI[ch] = Fi[i][1];
      FB[ch] = Fi[i][2];
      TA[ch] = Fi[0][i];
      TDI[ch] = Fi[1][i];
      TB[ch] = Fi[2][i];
    }
  }
  double* fA = facF + (long long)c * SR * mp;
  double* fT = facT ? facT + (long long)c * SR * mp : nullptr;
  auto put = [&](double* rec_row, const double (&val)[NCH]) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      if (k < mp) rec_row[k] = k < m ? val[ch] : 0.0;
    }
  };

  // level/flow coupling: XC = T^{-1} Ec, XR = T^{-T} Er^T, S3 = F - Er XC
  // (the flow lanes of the factor rows are zero here, so the sweeps of the
  // coupling columns leave zeros there)
  double EC[3][NCH], ER[3][NCH], XC[3][NCH], XR[3][NCH];
  if (arw) {
    const int PX = smw_arrow_row(g);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int k = ch * WAVE + lane;
        EC[i][ch] = k < L ? rc[(long long)(g.fa + i) * mp + k] : 0.0;
        ER[i][ch] = k < L ? rc[(long long)(g.fa + 3 + i) * mp + k] : 0.0;
      }
      smw_sweeps<double, NCH, false>(L, m, FA, FDI, FB, EC[i], 0.0, 0.0, 0.0, XC[i]);
      smw_sweeps<double, NCH, true>(L, m, TA, TDI, TB, ER[i], 0.0, 0.0, 0.0, XR[i]);
    }
    double S3[3][3], Si[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double sp = 0.0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) sp += ER[i][ch] * XC[j][ch];
        S3[i][j] = F[i][j] - wave_sum_u(sp);
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
        Si[i][j] = S3[r1][c1] * S3[r2][c2] - S3[r1][c2] * S3[r2][c1];
      }
    const double d3 = S3[0][0] * Si[0][0] + S3[0][1] * Si[1][0] + S3[0][2] * Si[2][0];
    double rn3 = 1.0;
    for (int i = 0; i < 3; ++i) rn3 *= fabs(S3[i][0]) + fabs(S3[i][1]) + fabs(S3[i][2]);
    if (!(fabs(d3) > 1e-14 * rn3)) bad = true;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      if (k >= L) {
        const int i = k - L < 3 ? k - L : 0;
        FA[ch] = Si[i][0] / d3;
        FDI[ch] = Si[i][1] / d3;
        FB[ch] = Si[i][2] / d3;
        TA[ch] = Si[0][i] / d3;
        TDI[ch] = Si[1][i] / d3;
        TB[ch] = Si[2][i] / d3;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      put(fA + (long long)(PX + i) * mp, XC[i]);
      put(fA + (long long)(PX + 3 + i) * mp, ER[i]);
      if (fT) {
        put(fT + (long long)(PX + i) * mp, XR[i]);
        put(fT + (long long)(PX + 3 + i) * mp, EC[i]);
      }
    }
  }
  put(fA + P_A * mp, FA);
  put(fA + P_DINV * mp, FDI);
  put(fA + P_B * mp, FB);
  if (fT) {
    put(fT + P_A * mp, TA);
    put(fT + P_DINV * mp, TDI);
    put(fT + P_B * mp, TB);
  }

  // SMW-1: W_j = A0^{-1} u_j
  double W[RDM][NCH], V[RDM][NCH];
  double vv = 0.0, ww = 0.0;
#pragma unroll
  for (int j = 0; j < RDM; ++j) {
    if (j >= rd) break;
    double U[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      const int kk = k < m ? k : m - 1;
      U[ch] = pair_u(j, kk);
      V[j][ch] = pair_v(j, kk);
    }
    smw_sweeps<double, NCH, false>(L, m, FA, FDI, FB, U, pair_u(j, L), pair_u(j, L + 1),
                                   pair_u(j, L + 2), W[j]);
    if (arw) arrow_schur<double, NCH>(L, m, FA, FDI, FB, XC, ER, W[j]);
    put(fA + (P_W + j) * mp, W[j]);
    put(fA + (P_W + rd + j) * mp, V[j]);
    double sv = 0.0, sw = 0.0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const bool in = ch * WAVE + lane < m;
      sv += in ? V[j][ch] * V[j][ch] : 0.0;
      sw += in ? W[j][ch] * W[j][ch] : 0.0;
    }
    vv += wave_sum_u(sv);
    ww += wave_sum_u(sw);
  }

  // SMW-2: C = I + V^T W.  Mc[i] = row i of [C | I] at column `lane`.
  double Mc[RDM];
#pragma unroll
  for (int i = 0; i < RDM; ++i) {
    Mc[i] = lane == rd + i ? 1.0 : 0.0;
    if (i >= rd) continue;
#pragma unroll
    for (int j = 0; j < RDM; ++j) {
      if (j >= rd) break;
      double s = 0.0;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        s += ch * WAVE + lane < m ? V[i][ch] * W[j][ch] : 0.0;
      const double cij = (i == j ? 1.0 : 0.0) + wave_sum_u(s);
      Mc[i] = lane == j ? cij : Mc[i];
    }
  }
  // the entries of V^T W carry rounding of order eps |V| |W|
  const double tol = 1e-12 * (1.0 + sqrt(vv * ww));
#pragma unroll
  for (int k = 0; k < RDM; ++k) {
    if (k >= rd) break;
    int p = k;
    double best = fabs(readlane(Mc[k], k));
#pragma unroll
    for (int i = k + 1; i < RDM; ++i) {
      if (i >= rd) break;
      const double a = fabs(readlane(Mc[i], k));
      if (a > best) {
        best = a;
        p = i;
      }
    }
    if (!(best > tol)) bad = true;
    // swap rows k and p (p >= k, wave-uniform)
    double rowp = Mc[k];
#pragma unroll
    for (int i = k + 1; i < RDM; ++i) rowp = i == p ? Mc[i] : rowp;
#pragma unroll
    for (int i = k + 1; i < RDM; ++i) Mc[i] = i == p ? Mc[k] : Mc[i];
    Mc[k] = rowp;
    Mc[k] *= 1.0 / readlane(Mc[k], k);
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      if (i == k || i >= rd) continue;
      const double f = readlane(Mc[i], k);
      Mc[i] -= f * Mc[k];
    }
  }
  // lane rd + j holds column j of C^{-1}
  if (lane >= rd && lane < 2 * rd) {
    double* ic = invC + (long long)c * rd * rd + (lane - rd);
#pragma unroll
    for (int i = 0; i < RDM; ++i)
      if (i < rd) ic[i * rd] = Mc[i];
  }

  if (fT) {  // transposed factors: A0^{-T} v_j and u_j
#pragma unroll
    for (int j = 0; j < RDM; ++j) {
      if (j >= rd) break;
      double WT[NCH], U[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int k = ch * WAVE + lane;
        U[ch] = pair_u(j, k < m ? k : m - 1);
      }
      smw_sweeps<double, NCH, true>(L, m, TA, TDI, TB, V[j], pair_v(j, L), pair_v(j, L + 1),
                                    pair_v(j, L + 2), WT);
      if (arw) arrow_schur<double, NCH>(L, m, TA, TDI, TB, XR, EC, WT);
      put(fT + (P_W + j) * mp, WT);
      put(fT + (P_W + rd + j) * mp, U);
    }
  }
  const unsigned long long anybad = __ballot(bad);
  if (anybad && lane == 0) atomicMin(status, c);
}

template <int RDM>
static hipError_t launch_setup_r(const Mesh& g, const double* rec, double* facF, double* facT,
                                 double* invC, int* status, hipStream_t s) {
  const int grid = (g.N + WPB - 1) / WPB;
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: hipLaunchKernelGGL((k_smw_setup<1, RDM>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, facF, facT, invC, status); break;
    case 2: hipLaunchKernelGGL((k_smw_setup<2, RDM>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, facF, facT, invC, status); break;
    case 3: hipLaunchKernelGGL((k_smw_setup<3, RDM>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, facF, facT, invC, status); break;
    case 4: hipLaunchKernelGGL((k_smw_setup<4, RDM>), dim3(grid), dim3(64 * WPB), 0, s, g, rec, facF, facT, invC, status); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_smw_setup(const Mesh& g, const double* rec, double* facF, double* facT,
                            double* invC, int* status, hipStream_t s) {
  if (band_walk(g)) return hipErrorInvalidValue;  // the band kernels serve those
  const int pw = smw_pairs(g);
  if (pw == 1) return launch_setup_r<1>(g, rec, facF, facT, invC, status, s);
  if (pw <= RANK_DIAG_MAX) return launch_setup_r<RANK_DIAG_MAX>(g, rec, facF, facT, invC, status, s);
  if (pw <= SMW_PAIRS_MAX) return launch_setup_r<SMW_PAIRS_MAX>(g, rec, facF, facT, invC, status, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- apply ----
// z = x0 - W C^{-1} (V^T x0) with x0 = A0^{-1} r (C^{-1} held by CapInv).
// One wavefront per CPW cells (the loads of all of them are issued before
// the first scan), NCH = ceil(m / 64) chunks of 64 unknowns held in
// registers, NR right-hand sides per launch starting at r0.  Scans and the
// reduction run on DPP lane moves; lanes past m read element m-1 and are
// masked.
#ifndef R1S_APPLY_CPW
#define R1S_APPLY_CPW 1
#endif
template <typename TV, int NCH, int NR, bool TRANS, int RDM, bool ARW>
__global__ __launch_bounds__(64 * WPB) void k_smw_apply(Mesh g, const TV* __restrict__ fac,
                                                       const TV* __restrict__ invC,
                                                       const double* __restrict__ rin,
                                                       double* __restrict__ zout, int r0) {
  constexpr int CPW = (NCH == 1 && RDM == 1) ? R1S_APPLY_CPW : 1;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = __builtin_amdgcn_readfirstlane((tile * WPB + (int)(threadIdx.x >> 6)) * CPW);
  if (c0 >= g.N) return;
  const int lane = lane_id();
  const int L = g.L, m = g.m;
  const long long mp = g.mp;
  const int rd = RDM == 1 ? 1 : smw_pairs(g);
  const int SR = smw_rows(g);
  const int PX = smw_arrow_row(g);
  constexpr int NX = ARW ? 3 : 1;
  TV A[CPW][NCH], DI[CPW][NCH], B[CPW][NCH], W[CPW][RDM][NCH], V[CPW][RDM][NCH];
  TV X[CPW][NX][NCH], E[CPW][NX][NCH];
  TV R[CPW][NR][NCH], RF[CPW][NR][3];
  CapInv<TV, RDM> IC[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = c0 + j < g.N ? c0 + j : g.N - 1;
    const TV* fc = fac + (long long)c * SR * mp;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      const int kk = k < m ? k : m - 1;
      A[j][ch] = ld_stream(fc + P_A * mp + kk);
      DI[j][ch] = ld_stream(fc + P_DINV * mp + kk);
      B[j][ch] = ld_stream(fc + P_B * mp + kk);
#pragma unroll
      for (int i = 0; i < RDM; ++i) {
        W[j][i][ch] = i < rd ? ld_stream(fc + (P_W + i) * mp + kk) : TV(0);
        V[j][i][ch] = i < rd ? ld_stream(fc + (P_W + rd + i) * mp + kk) : TV(0);
      }
      if constexpr (ARW) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          X[j][i][ch] = ld_stream(fc + (PX + i) * mp + kk);
          E[j][i][ch] = ld_stream(fc + (PX + 3 + i) * mp + kk);
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r)
        R[j][r][ch] = (TV)rin[(long long)(r0 + r) * g.n + (long long)c * m + kk];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        RF[j][r][i] = (TV)rin[(long long)(r0 + r) * g.n + (long long)c * m + L + i];
    IC[j].load(invC, c, rd, lane);
  }

#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = c0 + j;
    // several right-hand sides of a single-chunk cell share the coefficient
    // half of the sweeps' scans
    TV X0n[NR][NCH];
    if constexpr (NCH == 1 && NR > 1)
      smw_sweeps_nr<TV, NR, TRANS>(L, m, A[j][0], DI[j][0], B[j][0], R[j], RF[j], X0n);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      TV X0[NCH];
      if constexpr (NCH == 1 && NR > 1) {
        X0[0] = X0n[r][0];
      } else {
        smw_sweeps<TV, NCH, TRANS>(L, m, A[j], DI[j], B[j], R[j][r], RF[j][r][0], RF[j][r][1],
                                   RF[j][r][2], X0);
      }
      if constexpr (ARW) arrow_schur<TV, NCH>(L, m, A[j], DI[j], B[j], X[j], E[j], X0);
      TV s[RDM], z[RDM];
#pragma unroll
      for (int g0 = 0; g0 < RDM; g0 += 4) {  // wave sums four at a time
        TV s4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s4[e] = TV(0);
          if (g0 + e < RDM) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) s4[e] += V[j][g0 + e][ch] * X0[ch];
          }
        }
        wave_sums_u(s4);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (g0 + e < RDM) s[g0 + e] = g0 + e < rd ? s4[e] : TV(0);
      }
      IC[j].template apply<TRANS>(s, z, rd);
      if (c < g.N) {
        double* zv = zout + (long long)(r0 + r) * g.n + (long long)c * m;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const int k = ch * WAVE + lane;
          TV o = X0[ch];
#pragma unroll
          for (int i = 0; i < RDM; ++i) o -= z[i] * W[j][i][ch];
          if (k < m) st_out(zv + k, (double)o);
        }
      }
    }
  }
}

// Workgroup-per-cell form for m > 64: wave w owns unknowns 64w .. 64w+63.
// Each wave scans its chunk; the chunk compositions go through LDS and every
// wave folds in the compositions of the chunks before it (forward sweep) or
// after it (backward sweep), in a fixed order.
template <typename TV, int NCH, int NR, bool TRANS, int RDM, bool ARW>
__global__ __launch_bounds__(64 * NCH) void k_smw_apply_wg(Mesh g, const TV* __restrict__ fac,
                                                           const TV* __restrict__ invC,
                                                           const double* __restrict__ rin,
                                                           double* __restrict__ zout, int r0) {
  __shared__ TV fa[NR][NCH], fb[NR][NCH], ga[NR][NCH], gb[NR][NCH], ss[NR][RDM][NCH];
  constexpr int NX = ARW ? 3 : 1;
  __shared__ TV tt[NR][NX][NCH], zz[NR][NX];
  const int c = __builtin_amdgcn_readfirstlane(xcd_tile((int)blockIdx.x, (int)gridDim.x));
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const int L = g.L, m = g.m;
  const long long mp = g.mp;
  const int rd = RDM == 1 ? 1 : smw_pairs(g);
  const int SR = smw_rows(g);
  const int PX = smw_arrow_row(g);
  const int k = wv * WAVE + lane;
  const int kk = k < m ? k : m - 1;
  const bool lev = k < L;
  const bool has_lev = wv * WAVE < L;  // wave-uniform
  const TV* fc = fac + (long long)c * SR * mp;
  const TV A = ld_stream(fc + P_A * mp + kk);
  const TV DI = ld_stream(fc + P_DINV * mp + kk);
  const TV B = ld_stream(fc + P_B * mp + kk);
  TV W[RDM], V[RDM];
#pragma unroll
  for (int i = 0; i < RDM; ++i) {
    W[i] = i < rd ? ld_stream(fc + (P_W + i) * mp + kk) : TV(0);
    V[i] = i < rd ? ld_stream(fc + (P_W + rd + i) * mp + kk) : TV(0);
  }
  TV X[NX], E[NX];
  if constexpr (ARW) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      X[i] = ld_stream(fc + (PX + i) * mp + kk);
      E[i] = ld_stream(fc + (PX + 3 + i) * mp + kk);
    }
  }
  TV R[NR], RF[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double* rv = rin + (long long)(r0 + r) * g.n + (long long)c * m;
    R[r] = (TV)rv[kk];
    RF[r][0] = (TV)rv[L];
    RF[r][1] = (TV)rv[L + 1];
    RF[r][2] = (TV)rv[L + 2];
  }
  CapInv<TV, RDM> IC;
  IC.load(invC, c, rd, lane);

  TV a[NR], bb[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {  // forward sweep, local to the chunk
    a[r] = lev ? A : TV(0);
    bb[r] = lev ? (TRANS ? DI * R[r] : R[r]) : TV(0);
    if (has_lev) scan_affine_up_dpp(a[r], bb[r]);
    if (lane == WAVE - 1) {
      fa[r][wv] = a[r];
      fb[r][wv] = bb[r];
    }
  }
  __syncthreads();
  TV a2[NR], b2[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {  // carry in, then the backward sweep
    TV carry = TV(0);
    for (int w = 0; w < wv; ++w) carry = fb[r][w] + fa[r][w] * carry;
    const TV Y = bb[r] + a[r] * carry;
    a2[r] = lev ? B : TV(0);
    b2[r] = lev ? (TRANS ? Y : DI * Y) : TV(0);
    if (has_lev) scan_affine_down_dpp(a2[r], b2[r]);
    if (lane == 0) {
      ga[r][wv] = a2[r];
      gb[r][wv] = b2[r];
    }
  }
  __syncthreads();
  TV X0[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    TV carry = TV(0);
    for (int w = NCH - 1; w > wv; --w) carry = gb[r][w] + ga[r][w] * carry;
    const TV x0 = b2[r] + a2[r] * carry;
    const TV xf = A * RF[r][0] + DI * RF[r][1] + B * RF[r][2];
    X0[r] = lev ? x0 : (k < m ? xf : TV(0));
  }
  if constexpr (ARW) {  // the Schur step of the coupling, across the waves
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const TV tp = wave_sum_u(lev ? E[i] * X0[r] : TV(0));
        if (lane == 0) tt[r][i][wv] = tp;
      }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      TV t[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        t[i] = tt[r][i][0];
#pragma unroll
        for (int w = 1; w < NCH; ++w) t[i] += tt[r][i][w];
      }
      if (!lev && k < m) {
        X0[r] -= A * t[0] + DI * t[1] + B * t[2];
        zz[r][k - L] = X0[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (lev) X0[r] -= X[0] * zz[r][0] + X[1] * zz[r][1] + X[2] * zz[r][2];
  }
#pragma unroll
  for (int g0 = 0; g0 < NR * RDM; g0 += 4) {  // wave sums four at a time
    TV s4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      s4[e] = g0 + e < NR * RDM ? V[(g0 + e) % RDM] * X0[(g0 + e) / RDM] : TV(0);
    wave_sums_u(s4);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (g0 + e < NR * RDM && (g0 + e) % RDM < rd && lane == 0)
        ss[(g0 + e) / RDM][(g0 + e) % RDM][wv] = s4[e];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    TV s[RDM], z[RDM];
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      TV st = TV(0);
      if (i < rd) {
        st = ss[r][i][0];
#pragma unroll
        for (int w = 1; w < NCH; ++w) st += ss[r][i][w];
      }
      s[i] = st;
    }
    IC.template apply<TRANS>(s, z, rd);
    TV o = X0[r];
#pragma unroll
    for (int i = 0; i < RDM; ++i) o -= z[i] * W[i];
    if (k < m) st_out(zout + (long long)(r0 + r) * g.n + (long long)c * m + k, (double)o);
  }
}

// Right-hand sides per launch: 4 / 2 / 1 (2 / 1 with several diagonal pairs).
template <typename TV, int NCH, bool TRANS, int RDM, bool ARW>
static hipError_t launch_apply_t(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                 double* z, int nrhs, hipStream_t s) {
#ifndef R1S_NO_WG_CELL
  if constexpr (NCH > 1) {
    int r0 = 0;
    while (r0 < nrhs) {
      const int rem = nrhs - r0;
      // m > 128, one pair: a single right-hand side runs one wave per cell
      // over its chunks (no workgroup barrier; 249 us against 263 us for the
      // workgroup form at 512 x 256, m = 203)
      if (NCH > 2 && RDM == 1 && !ARW && rem == 1) {
        hipLaunchKernelGGL((k_smw_apply<TV, NCH, 1, TRANS, RDM, ARW>), dim3((g.N + WPB - 1) / WPB), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
        r0 += 1;
        continue;
      }
      if (RDM == 1 && rem >= 4) {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, RDM == 1 ? 4 : 2, TRANS, RDM, ARW>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += RDM == 1 ? 4 : 2;
      } else if (rem >= 2) {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, 2, TRANS, RDM, ARW>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += 2;
      } else {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, 1, TRANS, RDM, ARW>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += 1;
      }
    }
    return hipGetLastError();
  }
#endif
  constexpr int CPW = (NCH == 1 && RDM == 1) ? R1S_APPLY_CPW : 1;
  const int grid = (g.N + WPB * CPW - 1) / (WPB * CPW);
  int r0 = 0;
  while (r0 < nrhs) {
    const int rem = nrhs - r0;
    if constexpr (NCH == 1 && RDM == 1 && !ARW) {  // factors read once per 8 right-hand sides
      if (rem >= 8) {
        hipLaunchKernelGGL((k_smw_apply<TV, NCH, 8, TRANS, RDM, ARW>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
        r0 += 8;
        continue;
      }
    }
    if (RDM == 1 && rem >= 4) {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, RDM == 1 ? 4 : 2, TRANS, RDM, ARW>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += RDM == 1 ? 4 : 2;
    } else if (rem >= 2) {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, 2, TRANS, RDM, ARW>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, 1, TRANS, RDM, ARW>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += 1;
    }
  }
  return hipGetLastError();
}

template <typename TV, bool TRANS, int RDM, bool ARW>
static hipError_t launch_apply_nch(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                   double* z, int nrhs, hipStream_t s) {
  const int nch = (g.m + WAVE - 1) / WAVE;
  switch (nch) {
    case 1: return launch_apply_t<TV, 1, TRANS, RDM, ARW>(g, fac, invC, r, z, nrhs, s);
    case 2: return launch_apply_t<TV, 2, TRANS, RDM, ARW>(g, fac, invC, r, z, nrhs, s);
    case 3: return launch_apply_t<TV, 3, TRANS, RDM, ARW>(g, fac, invC, r, z, nrhs, s);
    case 4: return launch_apply_t<TV, 4, TRANS, RDM, ARW>(g, fac, invC, r, z, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TV, bool TRANS>
static hipError_t launch_apply_rank(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                    double* z, int nrhs, hipStream_t s) {
  if (g.rd > RANK_DIAG_MAX) return hipErrorInvalidValue;
  // level/flow coupling: one instantiation at the largest pair count (with
  // the atom's two terms beyond RANK_DIAG_MAX, a wider one)
  if (g.arrow) {
    if (smw_pairs(g) > RANK_DIAG_MAX)
      return launch_apply_nch<TV, TRANS, SMW_PAIRS_MAX, true>(g, fac, invC, r, z, nrhs, s);
    return launch_apply_nch<TV, TRANS, RANK_DIAG_MAX, true>(g, fac, invC, r, z, nrhs, s);
  }
  if (g.rd == 1) return launch_apply_nch<TV, TRANS, 1, false>(g, fac, invC, r, z, nrhs, s);
  return launch_apply_nch<TV, TRANS, RANK_DIAG_MAX, false>(g, fac, invC, r, z, nrhs, s);
}

hipError_t launch_smw_apply(const Mesh& g, const void* fac, const void* invC, bool f32, bool trans,
                            const double* r, double* z, int nrhs, hipStream_t s) {
  if (band_walk(g)) return hipErrorInvalidValue;
#ifndef R1S_NO_PACKED
  if (nrhs == 1 && packed_apply_ok(g))
    return launch_smw_apply_packed(g, fac, invC, f32, trans, r, z, 0, s);
#endif
  if (f32)
    return trans ? launch_apply_rank<float, true>(g, (const float*)fac, (const float*)invC, r, z, nrhs, s)
                 : launch_apply_rank<float, false>(g, (const float*)fac, (const float*)invC, r, z, nrhs, s);
  return trans ? launch_apply_rank<double, true>(g, (const double*)fac, (const double*)invC, r, z, nrhs, s)
               : launch_apply_rank<double, false>(g, (const double*)fac, (const double*)invC, r, z, nrhs, s);
}

}  // namespace r1s
