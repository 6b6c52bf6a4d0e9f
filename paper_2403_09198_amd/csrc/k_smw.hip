// Block-Jacobi preconditioner through the Sherman-Morrison-Woodbury identity.
//
// Section 6: the diagonal block of cell c is D_c = A0_c + u_cC v_cC^T with A0_c
// the sparse diagonal block of S.  With w = A0^{-1} u and C = 1 + v . w
// (SMW-1, SMW-2), D_c^{-1} r = x0 - w (v . x0) / C where x0 = A0^{-1} r.  The
// printed identity adds the correction; the correct Woodbury identity
// subtracts it, which is what is computed here.
//
// A0_c is the tridiagonal level band (no level/flow coupling) plus a dense
// 3 x 3 flow corner.  The band is factored once (LU without pivoting, the
// Thomas algorithm); each apply then runs the two bidiagonal sweeps as
// affine-map scans across the 64 lanes of one wavefront (a serial recurrence
// y_k = a_k y_{k-1} + b_k is a prefix composition of affine maps), carrying
// the last value from one 64-level chunk to the next.
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
// One thread per cell; runs once per matrix.  Factor records (see
// r1s_device.hpp): forward a = -l_k, dinv = 1/d_k, b = -s_k/d_k, w, v_cC;
// transpose a = -s_{k-1}/d_k, dinv, b = -l_{k+1}, wt = A0^{-T} v_cC, u_cC.
__global__ __launch_bounds__(256) void k_smw_setup(Mesh g, const double* __restrict__ rec,
                                                   double* __restrict__ facF,
                                                   double* __restrict__ facT,
                                                   double* __restrict__ invC, int* status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int L = g.L, m = g.m, mp = g.mp;
  const double* rc = rec + (long long)c * F_REC * mp;
  const double* dg = rc + (long long)F_DIAG * mp;
  const double* lo = rc + (long long)F_LO * mp;
  const double* hi = rc + (long long)F_HI * mp;
  const double* uC = rc + (long long)(F_U + D_C) * mp;
  const double* vC = rc + (long long)(F_V + D_C) * mp;
  double* fA = facF + (long long)c * F_SMW * mp;
  double* fT = facT ? facT + (long long)c * F_SMW * mp : nullptr;
  bool bad = false;

  for (int k = m; k < mp; ++k)
    for (int f = 0; f < F_SMW; ++f) {
      fA[f * mp + k] = 0.0;
      if (fT) fT[f * mp + k] = 0.0;
    }

  // LU of the level band: d_0 = a_0, l_k = sub_{k-1}/d_{k-1},
  // d_k = a_k - l_k sup_{k-1}.
  double dprev = 1.0;
  for (int k = 0; k < L; ++k) {
    const double l = k == 0 ? 0.0 : lo[k] / dprev;
    const double t = k == 0 ? 0.0 : l * hi[k - 1];
    const double d = dg[k] - t;
    if (!(fabs(d) > 1e-14 * (fabs(dg[k]) + fabs(t)))) bad = true;
    fA[P_A * mp + k] = -l;
    fA[P_DINV * mp + k] = 1.0 / d;
    dprev = d;
  }
  for (int k = 0; k < L; ++k) {
    const double di = fA[P_DINV * mp + k];
    fA[P_B * mp + k] = k <= L - 2 ? -hi[k] * di : 0.0;
    if (fT) {
      fT[P_A * mp + k] = k >= 1 ? -hi[k - 1] * di : 0.0;
      fT[P_DINV * mp + k] = di;
      fT[P_B * mp + k] = k <= L - 2 ? fA[P_A * mp + k + 1] : 0.0;
    }
  }

  // 3 x 3 flow corner, inverse by cofactors.
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
  if (!(fabs(det) > 1e-14 * rn)) bad = true;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Fi[i][j] /= det;
  for (int i = 0; i < 3; ++i) {
    fA[P_A * mp + L + i] = Fi[i][0];
    fA[P_DINV * mp + L + i] = Fi[i][1];
    fA[P_B * mp + L + i] = Fi[i][2];
    if (fT) {
      fT[P_A * mp + L + i] = Fi[0][i];
      fT[P_DINV * mp + L + i] = Fi[1][i];
      fT[P_B * mp + L + i] = Fi[2][i];
    }
  }

  // SMW-1: w = A0^{-1} u_cC (forward then backward sweep, then the corner).
  double* w = fA + P_W * mp;
  double prev = 0.0;
  for (int k = 0; k < L; ++k) {
    prev = uC[k] + fA[P_A * mp + k] * prev;
    w[k] = prev;
  }
  prev = 0.0;
  for (int k = L - 1; k >= 0; --k) {
    prev = fA[P_DINV * mp + k] * w[k] + fA[P_B * mp + k] * prev;
    w[k] = prev;
  }
  for (int i = 0; i < 3; ++i)
    w[L + i] = Fi[i][0] * uC[L] + Fi[i][1] * uC[L + 1] + Fi[i][2] * uC[L + 2];
  // SMW-2: capacitance C = 1 + v . w
  double vw = 0.0, vv = 0.0, ww = 0.0;
  for (int k = 0; k < m; ++k) {
    vw += vC[k] * w[k];
    vv += vC[k] * vC[k];
    ww += w[k] * w[k];
    fA[P_V * mp + k] = vC[k];
  }
  const double C = 1.0 + vw;
  if (!(fabs(C) > 1e-12 * (1.0 + sqrt(vv * ww)))) bad = true;
  invC[c] = 1.0 / C;

  if (fT) {  // wt = A0^{-T} v_cC, used by the transposed apply
    double* wt = fT + P_W * mp;
    prev = 0.0;
    for (int k = 0; k < L; ++k) {
      prev = fT[P_DINV * mp + k] * vC[k] + fT[P_A * mp + k] * prev;
      wt[k] = prev;
    }
    prev = 0.0;
    for (int k = L - 1; k >= 0; --k) {
      prev = wt[k] + fT[P_B * mp + k] * prev;
      wt[k] = prev;
    }
    for (int i = 0; i < 3; ++i)
      wt[L + i] = Fi[0][i] * vC[L] + Fi[1][i] * vC[L + 1] + Fi[2][i] * vC[L + 2];
    for (int k = 0; k < m; ++k) fT[P_V * mp + k] = uC[k];
  }
  if (bad) atomicMin(status, c);
}

hipError_t launch_smw_setup(const Mesh& g, const double* rec, double* facF, double* facT,
                            double* invC, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_smw_setup, dim3((g.N + 255) / 256), dim3(256), 0, s, g, rec, facF, facT,
                     invC, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- apply ----
// One wavefront per CPW cells (the loads of all of them are issued before
// the first scan), NCH = ceil(m / 64) chunks of 64 unknowns held in
// registers, NR right-hand sides per launch starting at r0.  Scans and the
// reduction run on DPP lane moves; lanes past m read element m-1 and are
// masked.
#ifndef R1S_APPLY_CPW
#define R1S_APPLY_CPW 1
#endif
template <typename TV, int NCH, int NR, bool TRANS>
__global__ __launch_bounds__(64 * WPB) void k_smw_apply(Mesh g, const TV* __restrict__ fac,
                                                       const TV* __restrict__ invC,
                                                       const double* __restrict__ rin,
                                                       double* __restrict__ zout, int r0) {
  constexpr int CPW = NCH == 1 ? R1S_APPLY_CPW : 1;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = __builtin_amdgcn_readfirstlane((tile * WPB + (int)(threadIdx.x >> 6)) * CPW);
  if (c0 >= g.N) return;
  const int lane = lane_id();
  const int L = g.L, m = g.m, mp = g.mp;
  TV A[CPW][NCH], DI[CPW][NCH], B[CPW][NCH], W[CPW][NCH], V[CPW][NCH];
  TV R[CPW][NR][NCH], RF[CPW][NR][3], IC[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = c0 + j < g.N ? c0 + j : g.N - 1;
    const TV* fc = fac + (long long)c * F_SMW * mp;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      const int kk = k < m ? k : m - 1;
      A[j][ch] = ld_stream(fc + P_A * mp + kk);
      DI[j][ch] = ld_stream(fc + P_DINV * mp + kk);
      B[j][ch] = ld_stream(fc + P_B * mp + kk);
      W[j][ch] = ld_stream(fc + P_W * mp + kk);
      V[j][ch] = ld_stream(fc + P_V * mp + kk);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        R[j][r][ch] = (TV)rin[(long long)(r0 + r) * g.n + (long long)c * m + kk];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        RF[j][r][i] = (TV)rin[(long long)(r0 + r) * g.n + (long long)c * m + L + i];
    IC[j] = invC[c];
  }

#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = c0 + j;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      TV Y[NCH];
      // forward sweep over the levels: y_k = a_k y_{k-1} + s1_k r_k
      TV carry = TV(0);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int k = ch * WAVE + lane;
        const bool lev = k < L;
        TV a = lev ? A[j][ch] : TV(0);
        TV bb = lev ? (TRANS ? DI[j][ch] * R[j][r][ch] : R[j][r][ch]) : TV(0);
        if (ch * WAVE < L) {
          scan_affine_up_dpp(a, bb);
          Y[ch] = bb + a * carry;
          carry = readlane(Y[ch], WAVE - 1);
        } else {
          Y[ch] = TV(0);
        }
      }
      // backward sweep: x_k = b_k x_{k+1} + s2_k y_k ; flow lanes: corner inverse
      carry = TV(0);
      TV s = TV(0);
      TV X0[NCH];
#pragma unroll
      for (int ch = NCH - 1; ch >= 0; --ch) {
        const int k = ch * WAVE + lane;
        const bool lev = k < L;
        TV a = lev ? B[j][ch] : TV(0);
        TV bb = lev ? (TRANS ? Y[ch] : DI[j][ch] * Y[ch]) : TV(0);
        TV x0;
        if (ch * WAVE < L) {
          scan_affine_down_dpp(a, bb);
          x0 = bb + a * carry;
          carry = readlane(x0, 0);
        } else {
          x0 = TV(0);
        }
        const TV xf = A[j][ch] * RF[j][r][0] + DI[j][ch] * RF[j][r][1] + B[j][ch] * RF[j][r][2];
        x0 = lev ? x0 : (k < m ? xf : TV(0));
        X0[ch] = x0;
        s += V[j][ch] * x0;
      }
      s = wave_sum_u(s) * IC[j];
      if (c < g.N) {
        double* zv = zout + (long long)(r0 + r) * g.n + (long long)c * m;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const int k = ch * WAVE + lane;
          if (k < m) zv[k] = (double)(X0[ch] - s * W[j][ch]);
        }
      }
    }
  }
}

// Workgroup-per-cell form for m > 64: wave w owns unknowns 64w .. 64w+63.
// Each wave scans its chunk; the chunk compositions go through LDS and every
// wave folds in the compositions of the chunks before it (forward sweep) or
// after it (backward sweep), in a fixed order.
template <typename TV, int NCH, int NR, bool TRANS>
__global__ __launch_bounds__(64 * NCH) void k_smw_apply_wg(Mesh g, const TV* __restrict__ fac,
                                                           const TV* __restrict__ invC,
                                                           const double* __restrict__ rin,
                                                           double* __restrict__ zout, int r0) {
  __shared__ TV fa[NR][NCH], fb[NR][NCH], ga[NR][NCH], gb[NR][NCH], ss[NR][NCH];
  const int c = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const int L = g.L, m = g.m, mp = g.mp;
  const int k = wv * WAVE + lane;
  const int kk = k < m ? k : m - 1;
  const bool lev = k < L;
  const bool has_lev = wv * WAVE < L;  // wave-uniform
  const TV* fc = fac + (long long)c * F_SMW * mp;
  const TV A = ld_stream(fc + P_A * mp + kk);
  const TV DI = ld_stream(fc + P_DINV * mp + kk);
  const TV B = ld_stream(fc + P_B * mp + kk);
  const TV W = ld_stream(fc + P_W * mp + kk);
  const TV V = ld_stream(fc + P_V * mp + kk);
  TV R[NR], RF[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double* rv = rin + (long long)(r0 + r) * g.n + (long long)c * m;
    R[r] = (TV)rv[kk];
    RF[r][0] = (TV)rv[L];
    RF[r][1] = (TV)rv[L + 1];
    RF[r][2] = (TV)rv[L + 2];
  }
  const TV ic = invC[c];

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
    const TV sp = wave_sum_u(V * X0[r]);
    if (lane == 0) ss[r][wv] = sp;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    TV st = ss[r][0];
#pragma unroll
    for (int w = 1; w < NCH; ++w) st += ss[r][w];
    st *= ic;
    if (k < m) zout[(long long)(r0 + r) * g.n + (long long)c * m + k] = (double)(X0[r] - st * W);
  }
}

template <typename TV, int NCH, bool TRANS>
static hipError_t launch_apply_t(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                 double* z, int nrhs, hipStream_t s) {
#ifndef R1S_NO_WG_CELL
  if constexpr (NCH > 1) {
    int r0 = 0;
    while (r0 < nrhs) {
      const int rem = nrhs - r0;
      if (rem >= 4) {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, 4, TRANS>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += 4;
      } else if (rem >= 2) {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, 2, TRANS>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += 2;
      } else {
        hipLaunchKernelGGL((k_smw_apply_wg<TV, NCH, 1, TRANS>), dim3(g.N), dim3(64 * NCH), 0, s, g, fac, invC, r, z, r0);
        r0 += 1;
      }
    }
    return hipGetLastError();
  }
#endif
  constexpr int CPW = NCH == 1 ? R1S_APPLY_CPW : 1;
  const int grid = (g.N + WPB * CPW - 1) / (WPB * CPW);
  int r0 = 0;
  while (r0 < nrhs) {
    const int rem = nrhs - r0;
    if (rem >= 4) {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, 4, TRANS>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += 4;
    } else if (rem >= 2) {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, 2, TRANS>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_smw_apply<TV, NCH, 1, TRANS>), dim3(grid), dim3(64 * WPB), 0, s, g, fac, invC, r, z, r0);
      r0 += 1;
    }
  }
  return hipGetLastError();
}

template <typename TV, bool TRANS>
static hipError_t launch_apply_nch(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                   double* z, int nrhs, hipStream_t s) {
  const int nch = (g.m + WAVE - 1) / WAVE;
  switch (nch) {
    case 1: return launch_apply_t<TV, 1, TRANS>(g, fac, invC, r, z, nrhs, s);
    case 2: return launch_apply_t<TV, 2, TRANS>(g, fac, invC, r, z, nrhs, s);
    case 3: return launch_apply_t<TV, 3, TRANS>(g, fac, invC, r, z, nrhs, s);
    case 4: return launch_apply_t<TV, 4, TRANS>(g, fac, invC, r, z, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_smw_apply(const Mesh& g, const void* fac, const void* invC, bool f32, bool trans,
                            const double* r, double* z, int nrhs, hipStream_t s) {
  if (f32)
    return trans ? launch_apply_nch<float, true>(g, (const float*)fac, (const float*)invC, r, z, nrhs, s)
                 : launch_apply_nch<float, false>(g, (const float*)fac, (const float*)invC, r, z, nrhs, s);
  return trans ? launch_apply_nch<double, true>(g, (const double*)fac, (const double*)invC, r, z, nrhs, s)
               : launch_apply_nch<double, false>(g, (const double*)fac, (const double*)invC, r, z, nrhs, s);
}

}  // namespace r1s
