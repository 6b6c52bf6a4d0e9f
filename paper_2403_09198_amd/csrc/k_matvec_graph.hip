// Packing and matvec on a general 2-D mesh: the block structure comes from
// the index arrays of the BR1-BSR format (section 5.1) instead of the
// structured 5-point stencil.  Each cell keeps the same per-cell record as on
// the structured mesh, with one neighbour slot per off-diagonal block of its
// block row (nbmax slots, at most 8) and explicit int32 tables: the neighbour
// cell of each slot and, for the transpose, the slot under which the
// neighbour lists this cell (block (nb, c) of the neighbour's record holds
// the transposed contribution; gathering it needs no atomics).
//
// y = J x (TRANS: J^T x), one wavefront per cell.  Phase 1 forms every pair
// coefficient of the block row (section 5.2: v . x_col per pair), phase 2
// streams the sparse rows and the output vectors of the pairs and writes y
// once.  Slots without a neighbour are skipped by wave-uniform branches, so
// a triangle cell (3 neighbours) reads only its own blocks.
#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

// ----------------------------------------------------------------- pack ----
// Record rows as on the structured mesh with graph slots: nbr rows
// F_NBR + s, pairs: the diagonal block's rd, then ro per slot.
template <typename TV>
__global__ __launch_bounds__(256) void k_pack_graph(Mesh g, GraphPackIn in, TV* __restrict__ rec) {
  const long long RS = (long long)g.F * g.mp;
  const long long total = (long long)g.N * RS;
  const int L = g.L, m = g.m, rd = g.rd, ro = g.ro, P = g.P;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / RS);
    const int rem = (int)(idx - (long long)c * RS);
    const int f = rem / g.mp, k = rem - f * g.mp;
    double val = 0.0;
    if (k < m) {
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
      } else if (f < g.fb) {
        const int s = f - F_NBR;
        if (g.nbr[(long long)c * g.nbmax + s] >= 0)
          val = in.s_nbr[(long long)(g.offb[c] + s) * m + k];
      } else if (f < g.fa) {
        const int t = f - g.fb, nbd = g.band - 1;
        const int j = (t < nbd ? t : t - nbd) + 2;
        const bool ok = k < L && (t < nbd ? k >= j : k + j < L);
        if (ok) val = in.s_band[((long long)c * 2 * nbd + t) * L + k];
      } else if (f < g.fu) {
        const int t = f - g.fa;
        if (k < L) val = (t < 3 ? in.s_lev_flow : in.s_flow_lev)[((long long)c * 3 + t % 3) * L + k];
      } else {
        const bool is_v = f >= g.fu + P;
        const int q = f - g.fu - (is_v ? P : 0);
        if (q < rd) {
          val = (is_v ? in.v_diag : in.u_diag)[((long long)c * rd + q) * m + k];
        } else {
          const int s = (q - rd) / ro, pp = (q - rd) - s * ro;
          if (g.nbr[(long long)c * g.nbmax + s] >= 0)
            val = (is_v ? in.v_off : in.u_off)[((long long)(g.offb[c] + s) * ro + pp) * m + k];
        }
      }
    }
    rec[idx] = (TV)val;
  }
}

hipError_t launch_pack_graph(const Mesh& g, const GraphPackIn& in, double* rec64, float* rec32,
                             hipStream_t s) {
  const long long total = (long long)g.N * g.F * g.mp;
  long long grid = (total + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_pack_graph<double>, dim3((unsigned)grid), dim3(256), 0, s, g, in, rec64);
  if (rec32) return launch_cast_f32(rec64, rec32, total, s);
  return hipGetLastError();
}

// --------------------------------------------------------------- matvec ----
// WIDE: further band diagonals or level/flow coupling in the diagonal block
// (the same terms as on the structured mesh).
template <typename TV, bool TRANS, bool RESID, bool WIDE>
__global__ __launch_bounds__(64 * WPB) void k_matvec_graph(Mesh g, const TV* __restrict__ rec,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ y, int r) {
  constexpr int RDM = RANK_DIAG_MAX, ROM = RANK_OFF_MAX, NBM = GRAPH_NBR_MAX;
  const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + (threadIdx.x >> 6)));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, L = g.L, rd = g.rd, ro = g.ro, P = g.P;
  const long long mp = g.mp, RS = (long long)g.F * mp;
  const int nch = (m + WAVE - 1) / WAVE;
  const TV* rc = rec + (long long)c * RS;
  const double* xr = x + (long long)r * g.n;
  const double* xc = xr + (long long)c * m;

  // slots: neighbour cell, the record holding the block, its rows
  int nb[NBM];
  const TV* base[NBM];
  int coef0[NBM], out0[NBM], nrow[NBM];
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    nb[s] = s < g.nbmax ? g.nbr[(long long)c * g.nbmax + s] : -1;
    const int t = (TRANS && nb[s] >= 0) ? g.tslot[(long long)c * g.nbmax + s] : s;
    base[s] = (TRANS && nb[s] >= 0) ? rec + (long long)nb[s] * RS : rc;
    coef0[s] = g.fu + (TRANS ? 0 : P) + rd + t * ro;
    out0[s] = g.fu + (TRANS ? P : 0) + rd + t * ro;
    nrow[s] = F_NBR + t;
  }
  const int dcoef0 = g.fu + (TRANS ? 0 : P), dout0 = g.fu + (TRANS ? P : 0);

  // phase 1: pair coefficients (partial sums per lane, then wave sums)
  TV pd[RDM], ps[NBM][ROM], as[3];
#pragma unroll
  for (int p = 0; p < RDM; ++p) pd[p] = TV(0);
#pragma unroll
  for (int s = 0; s < NBM; ++s)
#pragma unroll
    for (int p = 0; p < ROM; ++p) ps[s][p] = TV(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) as[i] = TV(0);
  for (int ch = 0; ch < nch; ++ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
    const bool in = k < m;
    const TV xk = in ? (TV)xc[kk] : TV(0);
#pragma unroll
    for (int p = 0; p < RDM; ++p)
      if (p < rd) pd[p] += rc[(dcoef0 + p) * mp + kk] * xk;
#pragma unroll
    for (int s = 0; s < NBM; ++s) {
      if (nb[s] < 0) continue;
      const TV xn = in ? (TV)xr[(long long)nb[s] * m + kk] : TV(0);
#pragma unroll
      for (int p = 0; p < ROM; ++p)
        if (p < ro) ps[s][p] += base[s][(coef0[s] + p) * mp + kk] * xn;
    }
    if (WIDE && g.arrow) {
#pragma unroll
      for (int i = 0; i < 3; ++i) as[i] += rc[(g.fa + (TRANS ? 0 : 3) + i) * mp + kk] * xk;
    }
  }
#pragma unroll
  for (int p = 0; p < RDM; ++p) pd[p] = p < rd ? wave_sum_u(pd[p]) : TV(0);
#pragma unroll
  for (int s = 0; s < NBM; ++s)
#pragma unroll
    for (int p = 0; p < ROM; ++p) ps[s][p] = (nb[s] >= 0 && p < ro) ? wave_sum_u(ps[s][p]) : TV(0);
  if (WIDE && g.arrow) {
#pragma unroll
    for (int i = 0; i < 3; ++i) as[i] = wave_sum_u(as[i]);
  }

  // phase 2: the row (column) of each unknown
  for (int ch = 0; ch < nch; ++ch) {
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
    TV ca, cb;
    if (!TRANS) {
      ca = rc[F_LO * mp + kk];
      cb = rc[F_HI * mp + kk];
    } else {
      const TV ta = rc[F_HI * mp + pa];
      const TV tb = rc[F_LO * mp + pb];
      ca = va ? ta : TV(0);
      cb = vb ? tb : TV(0);
    }
    TV t = rc[F_DIAG * mp + kk] * (TV)xc[kk] + ca * (TV)xc[pa] + cb * (TV)xc[pb];
#pragma unroll
    for (int p = 0; p < RDM; ++p)
      if (p < rd) t += rc[(dout0 + p) * mp + kk] * pd[p];
#pragma unroll
    for (int s = 0; s < NBM; ++s) {
      if (nb[s] < 0) continue;
      t += base[s][nrow[s] * mp + kk] * (TV)xr[(long long)nb[s] * m + kk];
#pragma unroll
      for (int p = 0; p < ROM; ++p)
        if (p < ro) t += base[s][(out0[s] + p) * mp + kk] * ps[s][p];
    }
    if constexpr (WIDE) {
      BandLane<TV, TRANS> bl;
      bl.load(g, rc, kk);
      t += bl.apply(g, xc);
      if (g.arrow) {
#pragma unroll
        for (int i = 0; i < 3; ++i) t += rc[(g.fa + (TRANS ? 3 : 0) + i) * mp + kk] * (TV)xc[L + i];
        const int fi = kk - L;
        t += fi == 0 ? as[0] : fi == 1 ? as[1] : fi == 2 ? as[2] : TV(0);
      }
    }
    const long long o = (long long)r * g.n + (long long)c * m + kk;
    st_out(y + o, RESID ? b[o] - (double)t : (double)t);
  }
}


// Single-chunk form (m <= 64) for meshes with at most NBM <= 4 neighbours
// per cell and the plain diagonal-block pattern: like the structured kernel,
// every load of the wave is issued before the first reduction.  Slots past
// a cell's degree read the cell's own record (valid addresses) and are
// masked out of the sums.
template <typename TV, bool TRANS, bool RESID, int NBM, int RDM, int ROM>
__global__ __launch_bounds__(64 * WPB) void k_matvec_graph1(Mesh g, const TV* __restrict__ rec,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ y, int r) {
  constexpr bool EXACT = RDM == 1 && ROM == 1;
  const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + (threadIdx.x >> 6)));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, L = g.L;
  const int rd = EXACT ? 1 : g.rd, ro = EXACT ? 1 : g.ro, P = rd + g.nbmax * ro;
  const long long mp = g.mp, RS = (long long)g.F * mp;
  const TV* rc = rec + (long long)c * RS;
  const double* xr = x + (long long)r * g.n;
  const int kk = lane < m ? lane : m - 1;
  const bool in = lane < m;

  bool ex[NBM];
  int nbc[NBM];
  const TV* base[NBM];
  int coef0[NBM], out0[NBM], nrow[NBM];
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    const int nb = s < g.nbmax ? g.nbr[(long long)c * g.nbmax + s] : -1;
    ex[s] = nb >= 0;
    nbc[s] = ex[s] ? nb : c;
    const int t = (TRANS && ex[s]) ? g.tslot[(long long)c * g.nbmax + s]
                                   : (s < g.nbmax ? s : g.nbmax - 1);
    base[s] = (TRANS && ex[s]) ? rec + (long long)nb * RS : rc;
    coef0[s] = g.fu + (TRANS ? 0 : P) + rd + t * ro;
    out0[s] = g.fu + (TRANS ? P : 0) + rd + t * ro;
    nrow[s] = F_NBR + t;
  }
  const int dcoef0 = g.fu + (TRANS ? 0 : P), dout0 = g.fu + (TRANS ? P : 0);

  // every load first
  TV pd[RDM], ud[RDM], ps[NBM][ROM], us[NBM][ROM], xn[NBM], nv[NBM];
#pragma unroll
  for (int p = 0; p < RDM; ++p) {
    pd[p] = p < rd ? ld_stream(rc + (dcoef0 + p) * mp + kk) : TV(0);
    ud[p] = p < rd ? ld_stream(rc + (dout0 + p) * mp + kk) : TV(0);
  }
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    xn[s] = (TV)xr[(long long)nbc[s] * m + kk];
    nv[s] = ld_stream(base[s] + nrow[s] * mp + kk);
#pragma unroll
    for (int p = 0; p < ROM; ++p) {
      ps[s][p] = p < ro ? ld_stream(base[s] + (coef0[s] + p) * mp + kk) : TV(0);
      us[s][p] = p < ro ? ld_stream(base[s] + (out0[s] + p) * mp + kk) : TV(0);
    }
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
  const double* xc = xr + (long long)c * m;
  const TV xk = (TV)xc[kk];  // the band / corner partners come from other lanes below
  const TV dg = ld_stream(rc + F_DIAG * mp + kk);
  TV ca, cb;
  if (!TRANS) {
    ca = ld_stream(rc + F_LO * mp + kk);
    cb = ld_stream(rc + F_HI * mp + kk);
  } else {
    const TV ta = rc[F_HI * mp + pa];
    const TV tb = rc[F_LO * mp + pb];
    ca = va ? ta : TV(0);
    cb = vb ? tb : TV(0);
  }
  __builtin_amdgcn_sched_barrier(0);

  const TV xa = __shfl(xk, pa, WAVE), xb = __shfl(xk, pb, WAVE);
  TV t = dg * xk + ca * xa + cb * xb;
#pragma unroll
  for (int p = 0; p < RDM; ++p) {
    const TV a = wave_sum_u(in ? pd[p] * xk : TV(0));
    t += ud[p] * a;
  }
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    if (ex[s]) t += nv[s] * xn[s];
#pragma unroll
    for (int p = 0; p < ROM; ++p) {
      const TV a = wave_sum_u(in ? ps[s][p] * xn[s] : TV(0));
      t += us[s][p] * (ex[s] ? a : TV(0));
    }
  }
  const long long o = (long long)r * g.n + (long long)c * m + kk;
  st_out(y + o, RESID ? b[o] - (double)t : (double)t);
}

template <typename TV, bool TRANS, bool RESID, int NBM>
static void launch_graph1(const Mesh& g, const TV* rec, const double* x, const double* b,
                          double* y, int r, hipStream_t s) {
  const dim3 grid((g.N + WPB - 1) / WPB), block(64 * WPB);
  if (g.rd == 1 && g.ro == 1)
    hipLaunchKernelGGL((k_matvec_graph1<TV, TRANS, RESID, NBM, 1, 1>), grid, block, 0, s, g, rec, x, b, y, r);
  else
    hipLaunchKernelGGL((k_matvec_graph1<TV, TRANS, RESID, NBM, RANK_DIAG_MAX, RANK_OFF_SMALL>), grid,
                       block, 0, s, g, rec, x, b, y, r);
}

template <typename TV, bool TRANS, bool RESID>
static hipError_t launch_graph_t(const Mesh& g, const TV* rec, const double* x, const double* b,
                                 double* y, int nrhs, hipStream_t s) {
  const dim3 grid((g.N + WPB - 1) / WPB), block(64 * WPB);
  const bool fast = !wide_pattern(g) && g.m <= WAVE && g.nbmax >= 1 && g.nbmax <= 4 &&
                    g.ro <= RANK_OFF_SMALL;
  for (int r = 0; r < nrhs; ++r) {
    if (fast && g.nbmax <= 3)
      launch_graph1<TV, TRANS, RESID, 3>(g, rec, x, b, y, r, s);
    else if (fast)
      launch_graph1<TV, TRANS, RESID, 4>(g, rec, x, b, y, r, s);
    else if (wide_pattern(g))
      hipLaunchKernelGGL((k_matvec_graph<TV, TRANS, RESID, true>), grid, block, 0, s, g, rec, x, b, y, r);
    else
      hipLaunchKernelGGL((k_matvec_graph<TV, TRANS, RESID, false>), grid, block, 0, s, g, rec, x, b, y, r);
  }
  return hipGetLastError();
}

hipError_t launch_matvec_graph(const Mesh& g, const void* rec, bool f32, bool trans,
                               const double* x, const double* b, double* y, int nrhs, bool resid,
                               hipStream_t s) {
  if (!ranks_supported(g.rd, g.ro) || g.band > BAND_MAX || g.nbmax > GRAPH_NBR_MAX)
    return hipErrorInvalidValue;
  if (resid) {
    const double* r = (const double*)rec;
    return trans ? launch_graph_t<double, true, true>(g, r, x, b, y, nrhs, s)
                 : launch_graph_t<double, false, true>(g, r, x, b, y, nrhs, s);
  }
  if (f32) {
    const float* r = (const float*)rec;
    return trans ? launch_graph_t<float, true, false>(g, r, x, nullptr, y, nrhs, s)
                 : launch_graph_t<float, false, false>(g, r, x, nullptr, y, nrhs, s);
  }
  const double* r = (const double*)rec;
  return trans ? launch_graph_t<double, true, false>(g, r, x, nullptr, y, nrhs, s)
               : launch_graph_t<double, false, false>(g, r, x, nullptr, y, nrhs, s);
}

}  // namespace r1s
