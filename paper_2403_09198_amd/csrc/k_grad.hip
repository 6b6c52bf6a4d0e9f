// Gradients of a loss through the linear solve J x_r = b_r.
//
// With lambda_r = J^{-T} dLoss/dx_r the matrix cotangent is -sum_r lambda_r x_r^T.
// For block (c, d) = S_{c,d} + u v^T this gives, without forming any dense
// block: the pattern entries of S, du = -sum_r lambda_r[c] (v . x_r[nb]) and
// dv = -sum_r x_r[nb] (u . lambda_r[c]).  One wavefront per cell; the
// coefficients v . x and u . lambda are wave reductions kept in LDS.
#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

constexpr int GRAD_MAX_RHS = 64;

__global__ __launch_bounds__(256) void k_grad(Mesh g, const double* __restrict__ rec,
                                              const double* __restrict__ lam,
                                              const double* __restrict__ x, int nrhs, GradOut o) {
  __shared__ double coef[4][2][5][GRAD_MAX_RHS];
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c = __builtin_amdgcn_readfirstlane(tile * 4 + wave);
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, mp = g.mp, L = g.L;
  const double* rc = rec + (long long)c * F_REC * mp;
  int nb[5];
  neighbours(g, c, nb);

  // alpha[d][r] = v_{c,d} . x_r[nb_d],  beta[d][r] = u_{c,d} . lambda_r[c]
  for (int r = 0; r < nrhs; ++r) {
    const double* lr = lam + (long long)r * g.n + (long long)c * m;
    for (int d = 0; d < 5; ++d) {
      double a = 0.0, b = 0.0;
      if (nb[d] >= 0) {
        const double* xn = x + (long long)r * g.n + (long long)nb[d] * m;
        for (int k = lane; k < m; k += WAVE) {
          a += rc[(F_V + d) * mp + k] * xn[k];
          b += rc[(F_U + d) * mp + k] * lr[k];
        }
      }
      a = wave_sum(a);
      b = wave_sum(b);
      if (lane == 0) {
        coef[wave][0][d][r] = a;
        coef[wave][1][d][r] = b;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  for (int k = lane; k < m; k += WAVE) {
    double gdiag = 0.0, glo = 0.0, ghi = 0.0, gnbr[5] = {0, 0, 0, 0, 0};
    double gu[5] = {0, 0, 0, 0, 0}, gv[5] = {0, 0, 0, 0, 0};
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
    for (int r = 0; r < nrhs; ++r) {
      const double* lr = lam + (long long)r * g.n + (long long)c * m;
      const double* xc = x + (long long)r * g.n + (long long)c * m;
      const double lk = lr[k];
      gdiag -= lk * xc[k];
      if (va) glo -= lk * xc[pa];
      if (vb) ghi -= lk * xc[pb];
      for (int d = 0; d < 5; ++d) {
        if (nb[d] < 0) continue;
        const double* xn = x + (long long)r * g.n + (long long)nb[d] * m;
        const double xk = xn[k];
        if (d != D_C) gnbr[d] -= lk * xk;
        gu[d] -= lk * coef[wave][0][d][r];
        gv[d] -= xk * coef[wave][1][d][r];
      }
    }
    o.s_diag[(long long)c * m + k] = gdiag;
    if (k < L) {
      if (k >= 1) o.s_sub[(long long)c * (L - 1) + k - 1] = glo;
      if (k <= L - 2) o.s_sup[(long long)c * (L - 1) + k] = ghi;
    } else {
      const int i = k - L;
      const int ja = (i + 2) % 3, jb = (i + 1) % 3;
      o.s_flow[(long long)c * 6 + i * 2 + (ja > i ? ja - 1 : ja)] = glo;
      o.s_flow[(long long)c * 6 + i * 2 + (jb > i ? jb - 1 : jb)] = ghi;
    }
    for (int d = 0; d < 5; ++d) {
      if (d != D_C) o.s_nbr[((long long)c * 4 + nbr_slot(d)) * m + k] = gnbr[d];
      o.u[((long long)c * 5 + d) * m + k] = gu[d];
      o.v[((long long)c * 5 + d) * m + k] = gv[d];
    }
  }
}

hipError_t launch_grad(const Mesh& g, const double* rec, const double* lam, const double* x,
                       int nrhs, const GradOut& out, hipStream_t s) {
  if (nrhs > GRAD_MAX_RHS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad, dim3((g.N + 3) / 4), dim3(256), 0, s, g, rec, lam, x, nrhs, out);
  return hipGetLastError();
}

}  // namespace r1s
