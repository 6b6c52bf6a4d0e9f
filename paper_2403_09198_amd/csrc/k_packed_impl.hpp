// Packed workgroup kernels and the tile maps of the cell kernels (templates;
// instantiated in k_packed.hip).
//
// Packed form, for one pair per block, tridiagonal level band and no
// level/flow coupling: a workgroup of NW waves holds Q = floor(64 NW / m)
// consecutive cells laid along the flat lane index, thread t holding unknown
// k = t - q m of cell c0 + q, q = t / m.  Lanes idle only past Q m, where a
// wave per 64-unknown chunk of a cell leaves ceil(m / 64) 64 - m idle (a
// quarter of the lanes at m = 203, nearly half at m = 35).
//
// Matvec (section 5.2): every lane issues all of its loads first (its v and
// u rows, the sparse rows, the x entries of the five blocks of its row).
// The pair coefficients v_d . x_nb(d) are sums over the lanes of one cell,
// which may share a wave with the next cell: each wave forms one masked wave
// sum per cell it touches (NS at most), the partials go to LDS, and lanes
// t < 5 Q add them per cell in wave order (a fixed order, so results are
// reproducible bit for bit).  The band and corner partners x[k-1], x[k+1],
// x[L + (i+1)%3], x[L + (i+2)%3] of the cell's own block come from an LDS
// copy of the block.
//
// SMW apply (section 6, SMW steps, sign corrected): the two bidiagonal
// sweeps are affine-map scans over the flat lanes.  The flow lanes of a
// cell, and lanes past Q m, hold the zero map, which cuts the recurrence
// between cells (the first level of a cell has no predecessor and the last
// none after it), so one unsegmented scan serves all the cells of a wave;
// the waves' compositions are chained through LDS as in the workgroup form.
// The Woodbury dot products v . x0 are segmented sums like the matvec's.
#pragma once
#include "k_matvec_impl.hpp"

namespace r1s {

constexpr int PK_MMIN = 32;  // smallest packed block size (a wave touches <= 3 cells)

// ------------------------------------------------------- packed helpers ----
// Cells touched by wave w: q_lo .. q_hi (q_hi < q_lo when none is active).
__device__ inline void pk_wave_cells(int w, int m, int qn, int& q_lo, int& q_hi) {
  q_lo = (w * WAVE) / m;
  const int hi = (w * WAVE + WAVE - 1) / m;
  q_hi = hi < qn - 1 ? hi : qn - 1;
}

// Sum of the partials of cell q over the waves that hold it, in wave order.
template <typename TV, int NS>
__device__ inline TV pk_cell_sum(const TV (*part)[NS], int q, int m) {
  const int w0 = (q * m) / WAVE, w1 = (q * m + m - 1) / WAVE;
  TV s = part[w0][q - (w0 * WAVE) / m];
  for (int w = w0 + 1; w <= w1; ++w) s += part[w][q - (w * WAVE) / m];
  return s;
}

// --------------------------------------------------------------- matvec ----
template <typename TV, int NW, int NS, bool TRANS, bool RESID, bool BAND>
__global__ __launch_bounds__(64 * NW) void k_matvec_pk(Mesh g_, const TV* __restrict__ rec,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ y, int Q, int r0) {
  constexpr int T = 64 * NW, QMAX = T / PK_MMIN;
  __shared__ TV part[5][NW][NS];
  __shared__ TV tot[5][QMAX];
  __shared__ TV xs[T];
  const Mesh g = kmesh<true>(g_);
  int c0, qn;
  cell_tile<BAND>(g, (int)blockIdx.x, Q, c0, qn);
  if (qn <= 0) return;  // the whole workgroup: no barrier is skipped by a part of it
  const int t = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = lane_id();
  const int m = g.m, L = g.L;
  const long long mp = g.mp;
  const int q = t / m;
  const bool act = q < qn;
  const int qq = act ? q : qn - 1;
  const int k = act ? t - q * m : m - 1;
  const int c = c0 + qq;
  int nb[5], nbc[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
  }
  CellRows<TV, TRANS> R;
  R.init(g, rec, c, nbc);
  const double* xr = x + (long long)r0 * g.n;

  TV pv[5], xv[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    pv[d] = ld_stream(R.base[d] + R.coef0[d] * mp + k);
    xv[d] = (TV)xr[(long long)nbc[d] * m + k];
  }
  int pa, pb;
  bool va, vb;
  if (k < L) {
    va = k >= 1; pa = va ? k - 1 : k;
    vb = k <= L - 2; pb = vb ? k + 1 : k;
  } else {
    const int i = k - L;
    pa = L + (i + 2) % 3; va = true;
    pb = L + (i + 1) % 3; vb = true;
  }
  const TV dg = ld_stream(R.rc + F_DIAG * mp + k);
  TV ca, cb;
  if (!TRANS) {
    ca = ld_stream(R.rc + F_LO * mp + k);
    cb = ld_stream(R.rc + F_HI * mp + k);
  } else {
    const TV ta = R.rc[F_HI * mp + pa];
    const TV tb = R.rc[F_LO * mp + pb];
    ca = va ? ta : TV(0);
    cb = vb ? tb : TV(0);
  }
  TV nv[5], uv[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C) nv[d] = ld_stream(R.base[d] + R.nbr[d] * mp + k);
    uv[d] = ld_stream(R.base[d] + R.out0[d] * mp + k);
  }
  __builtin_amdgcn_sched_barrier(0);
  xs[t] = xv[D_C];

  int q_lo, q_hi;
  pk_wave_cells(wv, m, qn, q_lo, q_hi);
#pragma unroll
  for (int g0 = 0; g0 < 5 * NS; g0 += 4) {  // multi-value wave sums, four at a time
    TV s4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int d = (g0 + e) / NS, j = (g0 + e) % NS;
      s4[e] = g0 + e < 5 * NS && act && q == q_lo + j ? pv[d] * xv[d] : TV(0);
    }
    wave_sums_u(s4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int d = (g0 + e) / NS, j = (g0 + e) % NS;
      if (g0 + e < 5 * NS && q_lo + j <= q_hi && lane == 0) part[d][wv][j] = s4[e];
    }
  }
  __syncthreads();
  if (t < 5 * qn) {
    const int d = t / qn, qc = t - d * qn;
    tot[d][qc] = pk_cell_sum<TV, NS>(part[d], qc, m);
  }
  __syncthreads();
  const int cb0 = qq * m;
  TV r = dg * xv[D_C] + ca * xs[cb0 + pa] + cb * xs[cb0 + pb];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C && ex[d]) r += nv[d] * xv[d];
    r += uv[d] * (ex[d] ? tot[d][qq] : TV(0));
  }
  if (act) {
    const long long o = (long long)r0 * g.n + (long long)c * m + k;
    st_out(y + o, RESID ? b[o] - (double)r : (double)r);
  }
}

// ------------------------------------------------------------ SMW apply ----
// Factor record rows as in the wave-per-cell apply: a, dinv, b, W, V (one
// pair); C^{-1} one value per cell.  Tiles: plain.
template <typename TV, int NW, int NS, bool TRANS>
__global__ __launch_bounds__(64 * NW) void k_smw_apply_pk(Mesh g, const TV* __restrict__ fac,
                                                         const TV* __restrict__ invC,
                                                         const double* __restrict__ rin,
                                                         double* __restrict__ zout, int Q,
                                                         int r0) {
  __shared__ TV fa[NW], fb[NW], ga[NW], gb[NW];
  __shared__ TV ss[NW][NS];
  const int c0 = (int)blockIdx.x * Q;
  const int qn = g.N - c0 < Q ? g.N - c0 : Q;
  const int t = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = lane_id();
  const int L = g.L, m = g.m;
  const long long mp = g.mp;
  const int SR = smw_rows(g);
  const int q = t / m;
  const bool act = q < qn;
  const int qq = act ? q : qn - 1;
  const int k = act ? t - q * m : m - 1;
  const int c = c0 + qq;
  const bool lev = act && k < L;
  const TV* fc = fac + (long long)c * SR * mp;
  const TV A = ld_stream(fc + P_A * mp + k);
  const TV DI = ld_stream(fc + P_DINV * mp + k);
  const TV B = ld_stream(fc + P_B * mp + k);
  const TV W = ld_stream(fc + (P_W + 0) * mp + k);
  const TV V = ld_stream(fc + (P_W + 1) * mp + k);
  const double* rv = rin + (long long)r0 * g.n + (long long)c * m;
  const TV R = (TV)rv[k];
  const TV RF0 = (TV)rv[L], RF1 = (TV)rv[L + 1], RF2 = (TV)rv[L + 2];
  const TV ic = invC[c];

  // forward sweep y_k = a_k y_{k-1} + (TRANS ? dinv_k r_k : r_k)
  TV a = lev ? A : TV(0);
  TV bb = lev ? (TRANS ? DI * R : R) : TV(0);
  scan_affine_up_dpp(a, bb);
  if (lane == WAVE - 1) {
    fa[wv] = a;
    fb[wv] = bb;
  }
  __syncthreads();
  TV carry = TV(0);
  for (int w = 0; w < wv; ++w) carry = fb[w] + fa[w] * carry;
  const TV Y = bb + a * carry;
  // backward sweep x_k = b_k x_{k+1} + (TRANS ? y_k : dinv_k y_k)
  TV a2 = lev ? B : TV(0);
  TV b2 = lev ? (TRANS ? Y : DI * Y) : TV(0);
  scan_affine_down_dpp(a2, b2);
  if (lane == 0) {
    ga[wv] = a2;
    gb[wv] = b2;
  }
  __syncthreads();
  carry = TV(0);
  for (int w = NW - 1; w > wv; --w) carry = gb[w] + ga[w] * carry;
  const TV x0 = b2 + a2 * carry;
  // flow lanes: row k - L of the 3 x 3 corner inverse times the flow entries
  const TV xf = A * RF0 + DI * RF1 + B * RF2;
  const TV X0 = lev ? x0 : (act ? xf : TV(0));

  // Woodbury: s = v . x0 per cell, z = x0 - (s / C) w
  int q_lo, q_hi;
  pk_wave_cells(wv, m, qn, q_lo, q_hi);
  const TV p = V * X0;
  {
    TV sums[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) sums[j] = q == q_lo + j ? p : TV(0);
    wave_sums_u(sums);
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (q_lo + j <= q_hi && lane == 0) ss[wv][j] = sums[j];
  }
  __syncthreads();
  const TV sc = pk_cell_sum<TV, NS>(ss, qq, m);
  const TV o = X0 - (sc * ic) * W;
  if (act) st_out(zout + (long long)r0 * g.n + (long long)c * m + k, (double)o);
}

}  // namespace r1s
