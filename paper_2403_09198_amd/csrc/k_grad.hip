// Gradients of a loss through the linear solve J x_r = b_r.
//
// With lambda_r = J^{-T} dLoss/dx_r the matrix cotangent is -sum_r lambda_r x_r^T.
// For block (c, d) = S_{c,d} + sum_p u_p v_p^T this gives, without forming
// any dense block: the pattern entries of S, du_p = -sum_r lambda_r[c]
// (v_p . x_r[nb]) and dv_p = -sum_r x_r[nb] (u_p . lambda_r[c]).  One
// wavefront per cell; the coefficients v_p . x and u_p . lambda are wave
// reductions kept in LDS ([wave][2][pair][rhs], sized at launch).  The same
// kernel serves the structured mesh (blocks S, W, C, E, N) and a general mesh
// (the diagonal block, then one block per neighbour slot).
#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

constexpr int GRAD_MAX_RHS = 64;
constexpr int GRAD_LDS_MAX = 64 * 1024;

// The blocks of cell c's row: direction codes and column cells (-1: none).
template <bool GRAPH>
struct RowBlocks {
  int n;
  int dir[GRAPH ? 1 + GRAPH_NBR_MAX : 5], cell[GRAPH ? 1 + GRAPH_NBR_MAX : 5];
  __device__ inline void init(const Mesh& g, int c) {
    if constexpr (GRAPH) {
      n = 1 + g.nbmax;
      dir[0] = D_C;
      cell[0] = c;
      for (int s = 0; s < GRAPH_NBR_MAX; ++s) {
        dir[1 + s] = GSLOT + s;
        cell[1 + s] = s < g.nbmax ? g.nbr[(long long)c * g.nbmax + s] : -1;
      }
    } else {
      n = 5;
      neighbours(g, c, cell);
      for (int d = 0; d < 5; ++d) dir[d] = d;
    }
  }
};

template <bool GRAPH, typename Out>
__global__ __launch_bounds__(256) void k_grad(Mesh g, const double* __restrict__ rec,
                                              const double* __restrict__ lam,
                                              const double* __restrict__ x, int nrhs, Out o) {
  extern __shared__ double coef_all[];
  const int wpg = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c = __builtin_amdgcn_readfirstlane(tile * wpg + wave);
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, mp = g.mp, L = g.L, P = g.P;
  double* alpha = coef_all + (long long)wave * 2 * P * nrhs;  // [P][nrhs]: v_q . x_r[nb]
  double* beta = alpha + (long long)P * nrhs;                  // [P][nrhs]: u_q . lambda_r[c]
  const double* rc = rec + (long long)c * g.F * mp;
  RowBlocks<GRAPH> rb;
  rb.init(g, c);

  for (int bi = 0; bi < rb.n; ++bi) {
    const int d = rb.dir[bi], nbc = rb.cell[bi];
    const int q0 = pair_start(g, d), cnt = pair_count(g, d);
    for (int p = 0; p < cnt; ++p) {
      const int q = q0 + p;
      const double* uq = rc + (long long)(g.fu + q) * mp;
      const double* vq = rc + (long long)(g.fu + P + q) * mp;
      for (int r = 0; r < nrhs; ++r) {
        double a = 0.0, b = 0.0;
        if (nbc >= 0) {
          const double* xn = x + (long long)r * g.n + (long long)nbc * m;
          const double* lr = lam + (long long)r * g.n + (long long)c * m;
          for (int k = lane; k < m; k += WAVE) {
            a += vq[k] * xn[k];
            b += uq[k] * lr[k];
          }
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
          alpha[q * nrhs + r] = a;
          beta[q * nrhs + r] = b;
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // general pattern of S_cc: one gradient per entry (i, j) of the pattern
  if constexpr (!GRAPH) {
    if (g.pat) {
      for (int e = lane; e < g.pnnz; e += WAVE) {
        const int i = g.perow[e], j = g.pecol[e];
        double ge = 0.0;
        for (int r = 0; r < nrhs; ++r) {
          const long long o0 = (long long)r * g.n + (long long)c * m;
          ge -= lam[o0 + i] * x[o0 + j];
        }
        o.s_cc[(long long)c * g.pnnz + e] = ge;
      }
    }
  }

  // sparse part
  for (int k = lane; k < m; k += WAVE) {
    double gdiag = 0.0, glo = 0.0, ghi = 0.0;
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
    for (int r = 0; r < nrhs && !g.pat; ++r) {
      const double* lr = lam + (long long)r * g.n + (long long)c * m;
      const double* xc = x + (long long)r * g.n + (long long)c * m;
      const double lk = lr[k];
      gdiag -= lk * xc[k];
      if (va) glo -= lk * xc[pa];
      if (vb) ghi -= lk * xc[pb];
    }
    if (!g.pat) {  // (a general pattern's entries are done above)
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
    }
    // diagonals of the off-diagonal blocks (zero for blocks outside the mesh)
    for (int bi = 0; bi < rb.n; ++bi) {
      const int d = rb.dir[bi], nbc = rb.cell[bi];
      if (d == D_C) continue;
      double gn = 0.0;
      if (nbc >= 0)
        for (int r = 0; r < nrhs; ++r)
          gn -= lam[(long long)r * g.n + (long long)c * m + k] *
                x[(long long)r * g.n + (long long)nbc * m + k];
      if constexpr (GRAPH) {
        if (nbc >= 0) o.s_nbr[(long long)(g.offb[c] + d - GSLOT) * m + k] = gn;
      } else {
        o.s_nbr[((long long)c * 4 + nbr_slot(d)) * m + k] = gn;
      }
    }
    // wide pattern: further level diagonals and the level/flow coupling
    // (zero in the slots outside the block)
    if (k < L && !g.pat) {
      const int nbd = g.band - 1;
      for (int j = 2; j <= g.band; ++j) {
        double glj = 0.0, guj = 0.0;
        for (int r = 0; r < nrhs; ++r) {
          const double* xc = x + (long long)r * g.n + (long long)c * m;
          const double lk = lam[(long long)r * g.n + (long long)c * m + k];
          if (k >= j) glj -= lk * xc[k - j];
          if (k + j < L) guj -= lk * xc[k + j];
        }
        o.s_band[((long long)c * 2 * nbd + j - 2) * L + k] = glj;
        o.s_band[((long long)c * 2 * nbd + nbd + j - 2) * L + k] = guj;
      }
      // coupling slot i: S[k][X_i] and S[X_i][k] with X_i = L + i, or the
      // atom a = L - 1 for slot 3 (entries k < a; index a is not one)
      const int ns = arrow_slots(g);
      for (int i = 0; i < ns; ++i) {
        const int xi = arrow_unknown(L, i);
        const bool on = i < 3 || k < L - 1;
        double glf = 0.0, gfl = 0.0;
        for (int r = 0; r < nrhs && on; ++r) {
          const double* xc = x + (long long)r * g.n + (long long)c * m;
          const double* lc = lam + (long long)r * g.n + (long long)c * m;
          glf -= lc[k] * xc[xi];
          gfl -= lc[xi] * xc[k];
        }
        o.s_lev_flow[((long long)c * ns + i) * L + k] = glf;
        o.s_flow_lev[((long long)c * ns + i) * L + k] = gfl;
      }
    }
  }

  // rank-one pairs (zero for the pairs of blocks outside the mesh)
  for (int bi = 0; bi < rb.n; ++bi) {
    const int d = rb.dir[bi], nbc = rb.cell[bi];
    const int q0 = pair_start(g, d), cnt = pair_count(g, d);
    if (GRAPH && nbc < 0) continue;  // no such block, no output slot
    for (int p = 0; p < cnt; ++p) {
      const int q = q0 + p;
      long long ou;  // element offset of the pair's gradient row
      if constexpr (GRAPH) {
        ou = d == D_C ? ((long long)c * g.rd + p) * m
                      : ((long long)(g.offb[c] + d - GSLOT) * g.ro + p) * m;
      } else {
        ou = ((long long)c * P + q) * m;
      }
      for (int k = lane; k < m; k += WAVE) {
        double gu = 0.0, gv = 0.0;
        if (nbc >= 0) {
          for (int r = 0; r < nrhs; ++r) {
            gu -= lam[(long long)r * g.n + (long long)c * m + k] * alpha[q * nrhs + r];
            gv -= x[(long long)r * g.n + (long long)nbc * m + k] * beta[q * nrhs + r];
          }
        }
        if constexpr (GRAPH) {
          (d == D_C ? o.u_diag : o.u_off)[ou + k] = gu;
          (d == D_C ? o.v_diag : o.v_off)[ou + k] = gv;
        } else {
          o.u[ou + k] = gu;
          o.v[ou + k] = gv;
        }
      }
    }
  }
}

template <bool GRAPH, typename Out>
static hipError_t launch_grad_t(const Mesh& g, const double* rec, const double* lam,
                                const double* x, int nrhs, const Out& out, hipStream_t s) {
  if (nrhs > GRAD_MAX_RHS) return hipErrorInvalidValue;
  const size_t per_wave = (size_t)2 * g.P * nrhs * sizeof(double);
  int wpg = 4;
  while (wpg > 1 && wpg * per_wave > GRAD_LDS_MAX) wpg >>= 1;
  if (wpg * per_wave > GRAD_LDS_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_grad<GRAPH, Out>), dim3((g.N + wpg - 1) / wpg), dim3(64 * wpg),
                     wpg * per_wave, s, g, rec, lam, x, nrhs, out);
  return hipGetLastError();
}

hipError_t launch_grad(const Mesh& g, const double* rec, const double* lam, const double* x,
                       int nrhs, const GradOut& out, hipStream_t s) {
  return launch_grad_t<false>(g, rec, lam, x, nrhs, out, s);
}

hipError_t launch_grad_graph(const Mesh& g, const double* rec, const double* lam, const double* x,
                             int nrhs, const GraphGradOut& out, hipStream_t s) {
  return launch_grad_t<true>(g, rec, lam, x, nrhs, out, s);
}

}  // namespace r1s
