// Matvec kernels of the structured mesh (included by the files that
// instantiate them; every instantiation lives in exactly one of those files).
#pragma once
#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

// ------------------------------------------------ per-cell row pointers ----
// The rows a cell's output depends on, per block direction d.  Forward: the
// cell's own record (v rows give the coefficients, u rows the output).
// Transpose: block (nb, opposite d) of the neighbour's record (its u rows give
// the coefficients, its v rows the output; its diagonal is symmetric).
template <typename TV, bool TRANS>
struct CellRows {
  const TV* rc;          // own record
  const TV* base[5];     // record holding the block of direction d
  int coef0[5], out0[5]; // first coefficient row, first output row
  int nbr[5];            // neighbour-diagonal row

  __device__ inline void init(const Mesh& g, const TV* rec, int c, const int (&nbc)[5]) {
    const long long RS = (long long)g.F * g.mp;
    rc = rec + (long long)c * RS;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      const int bd = TRANS ? opposite(d) : d;
      base[d] = TRANS ? rec + (long long)nbc[d] * RS : rc;
      coef0[d] = g.fu + (TRANS ? 0 : g.P) + pair_start(g, bd);
      out0[d] = g.fu + (TRANS ? g.P : 0) + pair_start(g, bd);
      nbr[d] = F_NBR + nbr_slot(bd == D_C ? 0 : bd);
    }
  }
};

// Kernel-side mesh: with one pair per block, band 1 and no coupling (EXACT)
// the counts become compile-time constants and all row offsets fold.
template <bool EXACT>
__device__ inline Mesh kmesh(Mesh g) {
  if (EXACT) {
    g.rd = 1; g.ro = 1; g.P = 5; g.band = 1; g.arrow = 0;
    g.fb = F_BAND; g.fa = F_BAND; g.fu = F_BAND; g.F = F_BAND + 10;
    g.graph = 0; g.nbmax = 4;
  }
  return g;
}

// --------------------------------------------------------------- matvec ----
// TV: value / accumulation type.  NCH = ceil(m / 64) chunks of 64 unknowns,
// NR right-hand sides per launch starting at rhs r0.  RESID: write b - J x.
//
// Every load of a wave is independent of the reductions, so all of them are
// issued before the first wait: missing neighbours (mesh boundary) read the
// cell's own, valid addresses and are masked out of the sums instead of
// being skipped by a branch.  Lanes past m read element m-1 and are masked.
// Pair slots past a block's count are skipped by wave-uniform guards.
// WIDE: the diagonal block has further band diagonals or level/flow coupling
// (1), or a general pattern (2: ELL rows with a column table and dense
// indices, see PatLane and the slot helpers).
// pair2: two neighbouring waves of a workgroup share a cell, the second
// taking right-hand sides r0 + NR .. r0 + 2 NR - 1 (the cell's rows come
// from HBM once and from L2 for the second wave; half the registers of one
// wave holding all 2 NR).
template <typename TV, int NCH, int NR, bool TRANS, bool RESID, int RDM, int ROM, int WIDE,
          bool SHARED = false>
__global__ __launch_bounds__(64 * WPB) void k_matvec(Mesh g_, const TV* __restrict__ rec,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ y, int r0_,
                                                     int pair2, int band) {
  constexpr bool EXACT = RDM == 1 && ROM == 1;
  constexpr int RM = RDM > ROM ? RDM : ROM;
  constexpr bool PRELOAD = NCH == 1;  // hold the sparse rows across the reduction
  const Mesh g = kmesh<EXACT>(g_);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int c;
  if (band) {  // column-band tiles of WPB (pair2: WPB / 2) cells
    int c0, qn;
    band_tile(g, (int)blockIdx.x, pair2 ? WPB / 2 : WPB, c0, qn);
    const int q = pair2 ? wv >> 1 : wv;
    if (q >= qn) return;
    c = c0 + q;
  } else {
    const int wid = xcd_tile(blockIdx.x, gridDim.x) * WPB + wv;
    c = pair2 ? wid >> 1 : wid;
    if (c >= g.N) return;
  }
  const int r0 = pair2 ? r0_ + (wv & 1) * NR : r0_;
  const int lane = lane_id();
  const int m = g.m, L = g.L;
  const long long mp = g.mp;
  int nb[5], nbc[5], cnt[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
    cnt[d] = pair_count(g, d);
  }
  CellRows<TV, TRANS> R;
  R.init(g, rec, c, nbc);
  const double* xr = x + (long long)r0 * g.n;

  TV pv[5][RM][NCH], xv[NR][5][NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
#pragma unroll
      for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
        pv[d][p][ch] = p < cnt[d] ? ld_mat<SHARED>(R.base[d] + (R.coef0[d] + p) * mp + kk) : TV(0);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        xv[r][d][ch] = (TV)xr[(long long)r * g.n + (long long)nbc[d] * m + kk];
    }
  }

  // sparse part of the row: diagonal, level band / flow corner partners,
  // neighbour diagonals, and the output rows of the pairs
  TV dg[NCH], ca[NCH], cb[NCH], nv[5][NCH], uv[5][RM][NCH], xa[NR][NCH], xb[NR][NCH];
  // WIDE, single chunk, many neighbour pairs: the coupling rows (summed over
  // the levels, and per lane) and the cell's flow unknowns are loaded with
  // everything else instead of after the pair sums (measured: 11% faster
  // with 6 pairs per neighbour block, 6% slower with 2).  Without coupling
  // the rows read are other rows of the record (distinct, always present)
  // and their values are discarded.
  constexpr bool PRE_ARROW = WIDE == 1 && PRELOAD && ROM > RANK_OFF_SMALL;
  constexpr int NA = PRE_ARROW ? ARROW_SLOTS_MAX : 1;
  constexpr int NSM = WIDE == 2 ? PAT_SLOTS_MAX : ARROW_SLOTS_MAX;
  const int nsl = WIDE == 2 ? g.ns : arrow_slots(g);  // coupling slots (wave-uniform)
  TV arw[NA][NCH], alw[NA][NCH], xfl[NR][NA];
  // single chunk: the band / corner partners x[pa], x[pb] of the cell's own
  // block come from the lanes that loaded them (a lane permutation) instead
  // of further loads
  constexpr bool SHUFFLE_X = PRELOAD && NCH == 1;
  int pa_s[NCH], pb_s[NCH];
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
    dg[ch] = ld_mat<SHARED>(R.rc + F_DIAG * mp + kk);
    if (!TRANS) {  // row k of S_cc: lo at column pa, hi at column pb
      ca[ch] = ld_mat<SHARED>(R.rc + F_LO * mp + kk);
      cb[ch] = ld_mat<SHARED>(R.rc + F_HI * mp + kk);
    } else {       // column k of S_cc: hi of row pa, lo of row pb
      const TV ta = R.rc[F_HI * mp + pa];
      const TV tb = R.rc[F_LO * mp + pb];
      ca[ch] = va ? ta : TV(0);
      cb[ch] = vb ? tb : TV(0);
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (d != D_C) nv[d][ch] = ld_mat<SHARED>(R.base[d] + R.nbr[d] * mp + kk);
#pragma unroll
      for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
        uv[d][p][ch] = p < cnt[d] ? ld_mat<SHARED>(R.base[d] + (R.out0[d] + p) * mp + kk) : TV(0);
    }
    pa_s[ch] = pa;
    pb_s[ch] = pb;
    if constexpr (!SHUFFLE_X) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double* xv_c = xr + (long long)r * g.n + (long long)c * m;
        xa[r][ch] = (TV)xv_c[pa];
        xb[r][ch] = (TV)xv_c[pb];
      }
    }
    if constexpr (PRE_ARROW) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const bool on = i < nsl;
        arw[i][ch] = ld_mat<SHARED>(R.rc + (on ? arrow_sum_row<TRANS>(g, i) : F_DIAG + i) * mp + kk);
        alw[i][ch] = ld_mat<SHARED>(R.rc + (on ? arrow_lane_row<TRANS>(g, i) : F_NBR + i % 3) * mp + kk);
#pragma unroll
        for (int r = 0; r < NR; ++r)
          xfl[r][i] = (TV)xr[(long long)r * g.n + (long long)c * m + arrow_unknown(L, i)];
      }
    }
  };
  if (PRELOAD) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) load_sparse(ch);
    // keep these loads in flight during the reductions (one memory round
    // trip per wave instead of two)
    __builtin_amdgcn_sched_barrier(0);
  }

  // pair coefficients: forward v_p . x_nb, transpose u_p(nb, opp d) . x_nb
  // (multi-value wave sums, four at a time)
  TV acc[NR][5][RM];
  constexpr int PER_R = RDM + 4 * ROM, NSUM = NR * PER_R;
#pragma unroll
  for (int g0 = 0; g0 < NSUM; g0 += 4) {
    TV s4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      TV s = TV(0);
      if (g0 + e < NSUM) {
        const int r = (g0 + e) / PER_R;
        int d, p;
        pair_index<RDM, ROM>((g0 + e) % PER_R, d, p);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
          if (ch * WAVE + lane < m) s += pv[d][p][ch] * xv[r][d][ch];
      }
      s4[e] = s;
    }
    wave_sums_u(s4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (g0 + e < NSUM) {
        const int r = (g0 + e) / PER_R;
        int d, p;
        pair_index<RDM, ROM>((g0 + e) % PER_R, d, p);
        acc[r][d][p] = ex[d] ? s4[e] : TV(0);
      }
    }
  }
  // coupling sums of the flow unknowns (and the atom) over the cell's levels
  TV asum[NR][NSM];
  if constexpr (WIDE) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < NSM; ++i) asum[r][i] = TV(0);
    if (nsl > 0) {
#pragma unroll
      for (int i = 0; i < NSM; ++i) {
        if (i >= nsl) break;
        TV ar[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const int k = ch * WAVE + lane;
          if constexpr (PRE_ARROW)
            ar[ch] = k < m ? arw[i][ch] : TV(0);
          else
            ar[ch] = k < m ? R.rc[slot_sum_row<WIDE, TRANS>(g, i) * mp + (k < m ? k : m - 1)] : TV(0);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          TV t = TV(0);
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) t += ar[ch] * xv[r][D_C][ch];
          asum[r][i] = wave_sum_u(t);
        }
      }
    }
  }

  // Lanes past m computed exactly what lane m-1 computes (all their indices
  // are clamped), so every lane stores to its clamped index: duplicate lanes
  // write identical values and no branch is needed around the stores.
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    if (!PRELOAD) load_sparse(ch);
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
    DiagLane<TV, TRANS, WIDE> bl;
    TV al[NSM];
#pragma unroll
    for (int i = 0; i < NSM; ++i) al[i] = TV(0);
    if constexpr (WIDE) {
      bl.load(g, R.rc, kk);
#pragma unroll
      for (int i = 0; i < NSM; ++i) {
        if (i >= nsl) break;
        if constexpr (PRE_ARROW)
          al[i] = alw[i][ch];
        else
          al[i] = R.rc[slot_lane_row<WIDE, TRANS>(g, i) * mp + kk];
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if constexpr (SHUFFLE_X) {
        xa[r][ch] = __shfl(xv[r][D_C][ch], pa_s[ch], WAVE);
        xb[r][ch] = __shfl(xv[r][D_C][ch], pb_s[ch], WAVE);
      }
      TV t = dg[ch] * xv[r][D_C][ch] + ca[ch] * xa[r][ch] + cb[ch] * xb[r][ch];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        if (d != D_C && ex[d]) t += nv[d][ch] * xv[r][d][ch];
#pragma unroll
        for (int p = 0; p < (d == D_C ? RDM : ROM); ++p) t += uv[d][p][ch] * acc[r][d][p];
      }
      if constexpr (WIDE) {
        const double* xc = xr + (long long)r * g.n + (long long)c * m;
        if constexpr (SHUFFLE_X)
          t += bl.apply_lanes(g, xv[r][D_C][ch]);
        else
          t += bl.apply(g, xc);
        if (nsl > 0) {
          // level lanes: coupling entries times the flow unknowns (and the
          // atom); flow lane L + i (atom lane L - 1): the coupling sum.  A
          // general pattern the same with its dense indices px.
#pragma unroll
          for (int i = 0; i < NSM; ++i) {
            if (i >= nsl) break;
            if constexpr (PRE_ARROW)
              t += al[i] * xfl[r][i];
            else if constexpr (SHUFFLE_X)
              t += al[i] * readlane(xv[r][D_C][ch], slot_x<WIDE>(g, i));
            else
              t += al[i] * (TV)xc[slot_x<WIDE>(g, i)];
          }
          if constexpr (WIDE == 2) {
#pragma unroll
            for (int i = 0; i < NSM; ++i) {
              if (i >= nsl) break;
              if (kk == g.px[i]) t += asum[r][i];
            }
          } else {
            const int fi = kk - L;
            t += fi == 0 ? asum[r][0] : fi == 1 ? asum[r][1] : fi == 2 ? asum[r][2] : TV(0);
            if (nsl > 3 && fi == -1) t += asum[r][3];
          }
        }
      }
      const long long o = (long long)(r0 + r) * g.n + (long long)c * m + kk;
      st_out(y + o, RESID ? b[o] - (double)t : (double)t);
    }
  }
}

// Workgroup-per-cell form for m > 64: wave w of the workgroup owns unknowns
// 64w .. 64w+63 of one cell, issues all of its loads at once (like the
// single-chunk kernel), and the pair coefficients are summed over the waves
// through LDS in a fixed order.
template <typename TV, int NCH, int NR, bool TRANS, bool RESID, int RDM, int ROM, int WIDE,
          bool BAND = false>
__global__ __launch_bounds__(64 * NCH) void k_matvec_wg(Mesh g_, const TV* __restrict__ rec,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ y, int r0) {
  constexpr bool EXACT = RDM == 1 && ROM == 1;
  constexpr int RM = RDM > ROM ? RDM : ROM;
  __shared__ TV part[NR][5][RM][NCH];
  constexpr int NSM = WIDE == 2 ? PAT_SLOTS_MAX : ARROW_SLOTS_MAX;
  __shared__ TV apart[WIDE ? NR : 1][NSM][NCH];
  __shared__ TV xs[NR][WAVE * NCH];  // the cell's own x block (band / corner partners)
  const Mesh g = kmesh<EXACT>(g_);
  int c0, qn;
  if (BAND) {
    band_tile(g, (int)blockIdx.x, 1, c0, qn);
    if (qn == 0) return;  // the whole workgroup
  } else {
    c0 = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  }
  const int c = __builtin_amdgcn_readfirstlane(c0);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const int m = g.m, L = g.L;
  const long long mp = g.mp;
  int nb[5], nbc[5], cnt[5];
  bool ex[5];
  neighbours(g, c, nb);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    ex[d] = nb[d] >= 0;
    nbc[d] = ex[d] ? nb[d] : c;
    cnt[d] = pair_count(g, d);
  }
  CellRows<TV, TRANS> R;
  R.init(g, rec, c, nbc);
  const double* xr = x + (long long)r0 * g.n;
  const int k = wv * WAVE + lane;
  const int kk = k < m ? k : m - 1;

  TV pv[5][RM], xv[NR][5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
#pragma unroll
    for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
      pv[d][p] = p < cnt[d] ? ld_stream(R.base[d] + (R.coef0[d] + p) * mp + kk) : TV(0);
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
  const TV dg = ld_stream(R.rc + F_DIAG * mp + kk);
  TV ca, cb;
  if (!TRANS) {
    ca = ld_stream(R.rc + F_LO * mp + kk);
    cb = ld_stream(R.rc + F_HI * mp + kk);
  } else {
    const TV ta = R.rc[F_HI * mp + pa];
    const TV tb = R.rc[F_LO * mp + pb];
    ca = va ? ta : TV(0);
    cb = vb ? tb : TV(0);
  }
  TV nv[5], uv[5][RM];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    if (d != D_C) nv[d] = ld_stream(R.base[d] + R.nbr[d] * mp + kk);
#pragma unroll
    for (int p = 0; p < (d == D_C ? RDM : ROM); ++p)
      uv[d][p] = p < cnt[d] ? ld_stream(R.base[d] + (R.out0[d] + p) * mp + kk) : TV(0);
  }
  __builtin_amdgcn_sched_barrier(0);
  // partners x[pa], x[pb] may sit in another wave's chunk: each wave puts
  // its chunk in LDS and reads them back after the barrier below
#pragma unroll
  for (int r = 0; r < NR; ++r) xs[r][k] = xv[r][D_C];

  {
    constexpr int PER_R = RDM + 4 * ROM, NSUM = NR * PER_R;
#pragma unroll
    for (int g0 = 0; g0 < NSUM; g0 += 4) {
      TV s4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s4[e] = TV(0);
        if (g0 + e < NSUM) {
          const int r = (g0 + e) / PER_R;
          int d, p;
          pair_index<RDM, ROM>((g0 + e) % PER_R, d, p);
          s4[e] = k < m ? pv[d][p] * xv[r][d] : TV(0);
        }
      }
      wave_sums_u(s4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (g0 + e < NSUM && lane == 0) {
          const int r = (g0 + e) / PER_R;
          int d, p;
          pair_index<RDM, ROM>((g0 + e) % PER_R, d, p);
          part[r][d][p][wv] = s4[e];
        }
      }
    }
  }
  // wide pattern: this chunk's share of the coupling sums, band terms
  DiagLane<TV, TRANS, WIDE> bl;
  TV al[NSM];
#pragma unroll
  for (int i = 0; i < NSM; ++i) al[i] = TV(0);
  const int nsl = WIDE == 2 ? g.ns : arrow_slots(g);
  if constexpr (WIDE) {
    if (nsl > 0) {
#pragma unroll
      for (int i = 0; i < NSM; ++i) {
        if (i >= nsl) break;
        const TV ar = k < m ? R.rc[slot_sum_row<WIDE, TRANS>(g, i) * mp + kk] : TV(0);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const TV s = wave_sum_u(ar * xv[r][D_C]);
          if (lane == 0) apart[r][i][wv] = s;
        }
        al[i] = R.rc[slot_lane_row<WIDE, TRANS>(g, i) * mp + kk];
      }
    }
    bl.load(g, R.rc, kk);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    TV t = dg * xv[r][D_C] + ca * xs[r][pa] + cb * xs[r][pb];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      if (d != D_C && ex[d]) t += nv[d] * xv[r][d];
#pragma unroll
      for (int p = 0; p < (d == D_C ? RDM : ROM); ++p) {
        TV s = part[r][d][p][0];
#pragma unroll
        for (int w = 1; w < NCH; ++w) s += part[r][d][p][w];
        t += uv[d][p] * (ex[d] ? s : TV(0));
      }
    }
    if constexpr (WIDE) {
      const double* xc = xr + (long long)r * g.n + (long long)c * m;
      t += bl.apply(g, xc);
      if (nsl > 0) {
#pragma unroll
        for (int i = 0; i < NSM; ++i) {
          if (i >= nsl) break;
          t += al[i] * (TV)xc[slot_x<WIDE>(g, i)];
        }
        int si = -1;
        if constexpr (WIDE == 2) {
#pragma unroll
          for (int i = 0; i < NSM; ++i)
            if (i < nsl && kk == g.px[i]) si = i;
        } else {
          const int fi = kk - L;
          si = fi >= 0 && fi < 3 ? fi : (nsl > 3 && fi == -1 ? 3 : -1);
        }
        if (si >= 0) {
          TV s = apart[r][si][0];
#pragma unroll
          for (int w = 1; w < NCH; ++w) s += apart[r][si][w];
          t += s;
        }
      }
    }
    const long long o = (long long)(r0 + r) * g.n + (long long)c * m + kk;
    st_out(y + o, RESID ? b[o] - (double)t : (double)t);
  }
}

template <typename TV, int NCH, bool TRANS, bool RESID, int RDM, int ROM, int WIDE>
inline void launch_mv_nch(const Mesh& g, const TV* rec, const double* x, const double* b,
                          double* y, int nrhs, hipStream_t s) {
  constexpr bool EXACT = RDM == 1 && ROM == 1;
#ifndef R1S_NO_WG_CELL
  if constexpr (NCH > 1) {
    int r0 = 0;
    while (r0 < nrhs) {
      const int rem = nrhs - r0;
      if constexpr (EXACT) {
        if (rem >= 4) {
          hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 4, TRANS, RESID, RDM, ROM, WIDE>), dim3(g.N),
                             dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
          r0 += 4;
          continue;
        }
      }
      if (rem >= 2) {
        hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 2, TRANS, RESID, RDM, ROM, WIDE>), dim3(g.N),
                           dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
        r0 += 2;
      } else {
        hipLaunchKernelGGL((k_matvec_wg<TV, NCH, 1, TRANS, RESID, RDM, ROM, WIDE>), dim3(g.N),
                           dim3(64 * NCH), 0, s, g, rec, x, b, y, r0);
        r0 += 1;
      }
    }
    return;
  }
#endif
  const int band = R1S_MV_BAND;
  const int grid = band ? band_grid(g, WPB) : (g.N + WPB - 1) / WPB;
  int r0 = 0;
  while (r0 < nrhs) {
    const int rem = nrhs - r0;
    if constexpr (NCH <= 2 && EXACT) {
      if (rem >= 8) {  // two waves per cell, four right-hand sides each
        // (256 x 128, L = 61: 145 us against 159 us for one wave with all
        // eight at 184 registers, 2 waves per SIMD; four waves of two: 175 us)
        const int grid2 = band ? band_grid(g, WPB / 2) : (2 * g.N + WPB - 1) / WPB;
        hipLaunchKernelGGL((k_matvec<TV, NCH, 4, TRANS, RESID, RDM, ROM, WIDE, true>),
                           dim3(grid2), dim3(64 * WPB), 0, s, g, rec, x, b, y, r0, 1, band);
        r0 += 8;
        continue;
      }
      if (rem >= 4) {
        hipLaunchKernelGGL((k_matvec<TV, NCH, 4, TRANS, RESID, RDM, ROM, WIDE>), dim3(grid),
                           dim3(64 * WPB), 0, s, g, rec, x, b, y, r0, 0, band);
        r0 += 4;
        continue;
      }
    }
    if (rem >= 2) {
      hipLaunchKernelGGL((k_matvec<TV, NCH, 2, TRANS, RESID, RDM, ROM, WIDE>), dim3(grid),
                         dim3(64 * WPB), 0, s, g, rec, x, b, y, r0, 0, band);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_matvec<TV, NCH, 1, TRANS, RESID, RDM, ROM, WIDE>), dim3(grid),
                         dim3(64 * WPB), 0, s, g, rec, x, b, y, r0, 0, band);
      r0 += 1;
    }
  }
}

template <typename TV, bool TRANS, bool RESID, int RDM, int ROM, int WIDE>
inline hipError_t launch_mv_r(const Mesh& g, const TV* rec, const double* x, const double* b,
                              double* y, int nrhs, hipStream_t s) {
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: launch_mv_nch<TV, 1, TRANS, RESID, RDM, ROM, WIDE>(g, rec, x, b, y, nrhs, s); break;
    case 2: launch_mv_nch<TV, 2, TRANS, RESID, RDM, ROM, WIDE>(g, rec, x, b, y, nrhs, s); break;
    case 3: launch_mv_nch<TV, 3, TRANS, RESID, RDM, ROM, WIDE>(g, rec, x, b, y, nrhs, s); break;
    case 4: launch_mv_nch<TV, 4, TRANS, RESID, RDM, ROM, WIDE>(g, rec, x, b, y, nrhs, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Kernel choice: one pair per block with the tridiagonal uncoupled diagonal
// block (all counts compile-time), any supported pair counts, or any pair
// counts with the wide diagonal-block pattern.
}  // namespace r1s
