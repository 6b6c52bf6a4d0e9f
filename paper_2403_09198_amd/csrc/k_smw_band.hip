// Block-Jacobi through the Sherman-Morrison-Woodbury identity for the wide
// diagonal-block pattern: a level band of half-width `band` > 1 and/or
// level/flow coupling (section 4, "Temporal Source Jacobian": transitions up
// to a threshold jump in the level index give a banded source Jacobian whose
// rows also depend on temperature).
//
// A0 = S_cc = [[B, E_c], [E_r, F]] with B the L x L level band, E_c the level
// rows' flow columns, E_r the flow rows' level columns and F the 3 x 3 flow
// corner.  LU without pivoting of B (the band stays the band: no fill), then
// the 3 x 3 Schur complement of the flow unknowns:
//   A0 = [[L_B, 0], [E_r U_B^{-1}, I]] [[U_B, L_B^{-1} E_c], [0, S3]],
//   S3 = F - (E_r U_B^{-1}) (L_B^{-1} E_c).
// The Woodbury correction with the diagonal block's pairs (section 6, eq.
// SMW, sign corrected) is then the same as for the tridiagonal pattern.
//
// A band solve is a serial recurrence of order `band`, so here a pair of
// lanes owns one cell and walks its levels (32 cells per wavefront) instead
// of one wave per cell with lane-parallel scans: the scan of an order-h
// recurrence costs O(h^3 log 64) per lane, the serial walk O(h) per level.
// The band factors are stored tile-interleaved and level-major, [tile of 32
// cells][k][row][lane], so each half of a wave reads one factor entry of 32
// consecutive cells as one contiguous 256-byte run, and the walk keeps the
// factor loads of the next levels in flight while it computes the current
// one (the recurrence itself only touches registers).  The Woodbury correction has no recurrence: a second
// kernel does it with one wavefront per cell on per-cell rows ([N][2 rd][mp]
// for W, V and [N][rd][rd] for C^{-1}), like the tridiagonal path.  With the
// atom density coupled to every molecule level (arrow = 2) the atom's column
// and row are two more Woodbury terms (rd + 2 in place of rd), as there.
// Right-hand sides and results keep the [nrhs][N][m] vector layout.
#include <math.h>

#include <type_traits>

#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

// Cells per general-pattern workgroup (one wavefront, one lane per cell).
constexpr int TILE = WAVE;
// Cells per band workgroup: the walk runs one wavefront per 32 cells, lanes
// c and c + 32 both on cell c (each loads half of a step's factor values, and
// one lane swap gives both lanes all of them), so that twice as many
// wavefronts stream factors as with one lane per cell.  The setup runs one
// lane per cell.
constexpr int BT = WAVE / 2;

// Row offsets of the band factors inside one tile of BT cells, stored
// level-major ([L][rows][BT]: the rows one step of a walk reads are adjacent,
// and the walk streams through the tile's factors in order):
//   lo(j) rows 0..band-1       l_{k,j} = L_B[k][k-j]      (k >= j)
//   ui     row band            1 / U_B[k][k]
//   up(j) rows band+1..2 band  U_B[k][k+j]                 (k + j < L)
//   ec(i) rows 2 band+1+i      (L_B^{-1} E_c)[k][i]        (coupling only)
//   er(i) rows 2 band+4+i      (E_r U_B^{-1})[i][k]        (coupling only)
__host__ __device__ inline int band_rows(const Mesh& g) { return 2 * g.band + 1 + (g.arrow ? 6 : 0); }
__host__ __device__ inline long long tiles(const Mesh& g) { return (g.N + TILE - 1) / TILE; }
__host__ __device__ inline long long band_tiles(const Mesh& g) { return (g.N + BT - 1) / BT; }


// ---------------------------------------------------------------- setup ----
// The factorisation, one lane per cell (workgroups of BT = one tile): the
// band factors and the Schur inverse (s3i [tile][9][BT]).  The Woodbury
// factors follow in the kernels below launch_band_solve: W and V rows for
// the forward apply (wv [N][2 rd][mp]: W_i = A0^{-1} u_i, then v_i) and,
// when wvT is given, for the transposed apply (A0^{-T} v_i, then u_i), and
// C^{-1} ([N][rd^2], row-major per cell).
__global__ __launch_bounds__(BT) void k_band_setup(Mesh g, const double* __restrict__ rec,
                                                     double* __restrict__ bf,
                                                     double* __restrict__ s3i_out, int* status) {
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int c = tile * BT + lane;
  if (c >= g.N) return;  // no cross-lane work in this kernel
  const int L = g.L, m = g.m, band = g.band;
  const long long mp = g.mp;
  const double* rc = rec + (long long)c * g.F * mp;
  const int RB = band_rows(g);
  double* fb = bf + (long long)tile * RB * L * BT + lane;
  auto F = [&](int row, int k) -> double& { return fb[((long long)k * RB + row) * BT]; };
  bool bad = false;

  // level band into the factor rows (lower j, diagonal, upper j)
  const int nbd = band - 1;
  for (int k = 0; k < L; ++k) {
    F(band, k) = rc[F_DIAG * mp + k];
    for (int j = 1; j <= band; ++j) {
      double lo = 0.0, up = 0.0;
      if (k >= j) lo = j == 1 ? rc[F_LO * mp + k] : rc[(g.fb + j - 2) * mp + k];
      if (k + j < L) up = j == 1 ? rc[F_HI * mp + k] : rc[(g.fb + nbd + j - 2) * mp + k];
      F(j - 1, k) = lo;
      F(band + j, k) = up;
    }
  }
  // band LU without pivoting, in place: for pivot k, rows i = k+1..k+band
  for (int k = 0; k < L; ++k) {
    const double piv = F(band, k);
    if (!(fabs(piv) > 1e-14 * fabs(rc[F_DIAG * mp + k]))) bad = true;
    const double inv = 1.0 / piv;
    for (int i = k + 1; i <= k + band && i < L; ++i) {
      const int ji = i - k;
      const double l = F(ji - 1, i) * inv;
      F(ji - 1, i) = l;
      for (int t = 1; t <= band && k + t < L; ++t) {
        const int col = k + t, dcol = col - i;  // column relative to row i
        const double u = F(band + t, k);
        if (dcol < 0) F(-dcol - 1, i) -= l * u;
        else if (dcol == 0) F(band, i) -= l * u;
        else if (dcol <= band) F(band + dcol, i) -= l * u;
      }
    }
  }
  // flow corner and its Schur complement
  double Fm[3][3];
  for (int i = 0; i < 3; ++i) {
    Fm[i][i] = rc[F_DIAG * mp + L + i];
    Fm[i][(i + 2) % 3] = rc[F_LO * mp + L + i];
    Fm[i][(i + 1) % 3] = rc[F_HI * mp + L + i];
  }
  if (g.arrow) {
    // E_c' = L_B^{-1} E_c (column i), E_r' = E_r U_B^{-1} (row i)
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < L; ++k) {
        double y = rc[(g.fa + i) * mp + k];
        for (int j = 1; j <= band && j <= k; ++j) y -= F(j - 1, k) * F(2 * band + 1 + i, k - j);
        F(2 * band + 1 + i, k) = y;
        double z = rc[(g.fa + 3 + i) * mp + k];
        for (int j = 1; j <= band && j <= k; ++j) z -= F(band + j, k - j) * F(2 * band + 4 + i, k - j);
        F(2 * band + 4 + i, k) = z / F(band, k);
      }
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int k = 0; k < L; ++k) s += F(2 * band + 4 + a, k) * F(2 * band + 1 + b, k);
        Fm[a][b] -= s;
      }
  }
  double Fi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
      Fi[i][j] = Fm[r1][c1] * Fm[r2][c2] - Fm[r1][c2] * Fm[r2][c1];
    }
  const double det = Fm[0][0] * Fi[0][0] + Fm[0][1] * Fi[1][0] + Fm[0][2] * Fi[2][0];
  double rn = 1.0;
  for (int i = 0; i < 3; ++i) rn *= fabs(Fm[i][0]) + fabs(Fm[i][1]) + fabs(Fm[i][2]);
  if (!(fabs(det) > 1e-14 * rn)) bad = true;
  double s3i[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s3i[3 * i + j] = Fi[i][j] / det;
  for (int t = 0; t < 9; ++t) s3i_out[((long long)tile * 9 + t) * BT + lane] = s3i[t];
  for (int k = 0; k < L; ++k) F(band, k) = 1.0 / F(band, k);

  if (bad) atomicMin(status, c);
}

// The Woodbury terms of a cell, term i at element k: the block's pairs, then
// the atom's column (u = column, v = e_a) and row (u = e_a, v = row).
struct BandPairs {
  const double *rc, *uC, *vC;
  long long mp;
  int rdu, ia, colrow, rowrow;
  __device__ BandPairs(const Mesh& g, const double* rec, int c) {
    mp = g.mp;
    rc = rec + (long long)c * g.F * mp;
    uC = rc + (long long)(g.fu + pair_start(g, D_C)) * mp;
    vC = rc + (long long)(g.fu + g.P + pair_start(g, D_C)) * mp;
    rdu = g.rd;
    ia = g.L - 1;
    colrow = g.arrow == 2 ? arrow_col_row(g, 3) : 0;
    rowrow = g.arrow == 2 ? arrow_row_row(g, 3) : 0;
  }
  __device__ double u(int i, int k) const {
    if (i < rdu) return uC[i * mp + k];
    if (i == rdu) return k < ia ? rc[colrow * mp + k] : 0.0;
    return k == ia ? 1.0 : 0.0;
  }
  __device__ double v(int i, int k) const {
    if (i < rdu) return vC[i * mp + k];
    if (i == rdu) return k == ia ? 1.0 : 0.0;
    return k < ia ? rc[rowrow * mp + k] : 0.0;
  }
};

// The rows of wv before the solves, one wavefront per cell: row i = u_i (the
// right-hand side of W_i = A0^{-1} u_i, solved in place), row rd + i = v_i;
// wvT: v_i (for A0^{-T} v_i), then u_i.  Padding zeroed.
__global__ __launch_bounds__(64 * WPB) void k_band_wv_init(Mesh g, const double* __restrict__ rec,
                                                           double* __restrict__ wv,
                                                           double* __restrict__ wvT) {
  const int c = blockIdx.x * WPB + (int)(threadIdx.x >> 6);
  if (c >= g.N) return;
  const int lane = lane_id(), m = g.m, rd = smw_pairs(g);
  const long long mp = g.mp;
  const BandPairs pr(g, rec, c);
  double* w = wv + (long long)c * 2 * rd * mp;
  double* wt = wvT ? wvT + (long long)c * 2 * rd * mp : nullptr;
  for (int i = 0; i < rd; ++i)
    for (int k = lane; k < mp; k += WAVE) {
      const double u = k < m ? pr.u(i, k) : 0.0, v = k < m ? pr.v(i, k) : 0.0;
      w[i * mp + k] = u;
      w[(rd + i) * mp + k] = v;
      if (wt) {
        wt[i * mp + k] = v;
        wt[(rd + i) * mp + k] = u;
      }
    }
}

// C = I + V^T W of a cell (the W_i solved in place in wv) and its inverse,
// one wavefront per cell: the rd^2 dot products as multi-value wave sums,
// then Gauss-Jordan with partial pivoting on [C | I], lane t holding column t
// of the augmented matrix (pivots read with v_readlane, every step
// wave-uniform).  The transposed apply uses (C^{-1})^T.
template <int NCH>
__global__ __launch_bounds__(64 * WPB) void k_band_cinv(Mesh g, const double* __restrict__ wv,
                                                        double* __restrict__ cinv, int* status) {
  constexpr int RDM = SMW_PAIRS_MAX;
  const int c = blockIdx.x * WPB + (int)(threadIdx.x >> 6);
  if (c >= g.N) return;
  const int lane = lane_id(), m = g.m, rd = smw_pairs(g);
  const long long mp = g.mp;
  const double* w = wv + (long long)c * 2 * rd * mp;
  double V[RDM][NCH], W[RDM][NCH];
  double vv = 0.0, ww = 0.0;
#pragma unroll
  for (int i = 0; i < RDM; ++i)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      const bool in = i < rd && k < m;
      V[i][ch] = in ? w[(rd + i) * mp + k] : 0.0;
      W[i][ch] = in ? w[i * mp + k] : 0.0;
      vv += V[i][ch] * V[i][ch];
      ww += W[i][ch] * W[i][ch];
    }
  double Mc[RDM];  // row i of [C | I] at column `lane`
#pragma unroll
  for (int i = 0; i < RDM; ++i) Mc[i] = lane == rd + i ? 1.0 : 0.0;
  // C[i][j] = delta_ij + V_i . W_j, the sums of column j four at a time
  // (fixed trip counts and guards in place of early exits: every index is
  // a compile-time constant, so Mc stays in registers)
#pragma unroll
  for (int j = 0; j < RDM; ++j) {
    if (j < rd) {
#pragma unroll
      for (int g0 = 0; g0 < RDM; g0 += 4) {
        double s4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s4[e] = 0.0;
          if (g0 + e < RDM) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) s4[e] += V[g0 + e][ch] * W[j][ch];
          }
        }
        wave_sums_u(s4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = g0 + e;
          if (i < RDM && i < rd) Mc[i] = lane == j ? (i == j ? 1.0 : 0.0) + s4[e] : Mc[i];
        }
      }
    }
  }
  double t2[2] = {vv, ww};
  wave_sums_u(t2);
  // the entries of V^T W carry rounding of order eps |V| |W|
  const double tol = 1e-12 * (1.0 + sqrt(t2[0] * t2[1]));
  bool bad = false;
#pragma unroll
  for (int k = 0; k < RDM; ++k) {
    if (k < rd) {
      int p = k;
      double best = fabs(readlane(Mc[k], k));
#pragma unroll
      for (int i = k + 1; i < RDM; ++i) {
        const double a = i < rd ? fabs(readlane(Mc[i], k)) : 0.0;
        p = a > best ? i : p;
        best = a > best ? a : best;
      }
      if (!(best > tol)) bad = true;
      double rowp = Mc[k];  // swap rows k and p (p >= k, wave-uniform)
#pragma unroll
      for (int i = k + 1; i < RDM; ++i) rowp = i == p ? Mc[i] : rowp;
#pragma unroll
      for (int i = k + 1; i < RDM; ++i) Mc[i] = i == p ? Mc[k] : Mc[i];
      Mc[k] = rowp;
      Mc[k] *= 1.0 / readlane(Mc[k], k);
#pragma unroll
      for (int i = 0; i < RDM; ++i) {
        if (i != k && i < rd) {
          const double f = readlane(Mc[i], k);
          Mc[i] -= f * Mc[k];
        }
      }
    }
  }
  if (lane >= rd && lane < 2 * rd) {  // lane rd + j holds column j of C^{-1}
    double* ic = cinv + (long long)c * rd * rd + (lane - rd);
#pragma unroll
    for (int i = 0; i < RDM; ++i)
      if (i < rd) ic[i * rd] = Mc[i];
  }
  if (bad && lane == 0) atomicMin(status, c);
}

// ---------------------------------------------------------------- apply ----
// Software-pipelined walk: the loads of block b + 1 (U steps, one call of
// load(b + 1, steps)) are issued before block b is computed, and the walk
// runs whole pairs of blocks, so nothing in the loop is conditional: steps
// past the end are dead steps that the load and compute functions turn into
// no-ops (zero coefficients, a scratch slot for their result).  With no load
// or store under a branch, the compiler waits for exactly the loads of the
// block being computed.
template <int U, typename Step, typename LoadF, typename CompF>
__device__ __forceinline__ void pipelined_walk(int count, LoadF load, CompF comp) {
  Step A[U], B[U];
  auto ld = [&](int b, Step(&S)[U]) { load(b, S); };
  auto cp = [&](int b, Step(&S)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) comp(b * U + u, S[u]);
  };
  const int nb = (count + U - 1) / U;
  ld(0, A);
  for (int b = 0; b < nb; b += 2) {
    ld(b + 1, B);
    cp(b, A);
    ld(b + 2, A);
    cp(b + 1, B);
  }
}

// Ring walk: U steps in flight in U register slots.  Step k is computed from
// slot k % U, and the slot is refilled at once with the loads of step k + U,
// so that while one step is computed the loads of the next U - 1 are
// outstanding (the block walk above keeps only U in flight with 2 U slots).
// Vector loads return in order, so the wait before each step is for its own
// slot only; U is chosen so that the U - 1 steps outstanding stay within the
// 63 vector loads a wave can have in flight.  Steps past `count` are neither
// loaded nor computed (the last refill and the last block test the step).
template <int U, typename Step, typename LoadF, typename CompF>
__device__ __forceinline__ void ring_walk(int count, LoadF load, CompF comp) {
  Step S[U];
#pragma unroll
  for (int u = 0; u < U; ++u) load(u, S[u]);
  const int nb = (count + U - 1) / U;
  for (int b = 0; b < nb - 2; ++b) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      comp(b * U + u, S[u]);
      load((b + 1) * U + u, S[u]);
    }
  }
  if (nb >= 2) {  // the last refill loads only the steps that exist
#pragma unroll
    for (int u = 0; u < U; ++u) {
      comp((nb - 2) * U + u, S[u]);
      if ((nb - 1) * U + u < count) load((nb - 1) * U + u, S[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if ((nb - 1) * U + u < count) comp((nb - 1) * U + u, S[u]);
}

// x0 = A0^{-1} r (TRANS: A0^{-T} r) for one cell, in place in the cell's
// vector v[0..m) (v[m] is a scratch slot): the forward sweep (L_B y = r;
// TRANS: U_B^T y = r) with the coupling sums on the way, the 3 x 3 Schur
// inverse s3i (row major) on the flow unknowns, then the backward sweep
// (U_B x = y - E_c' x_f; TRANS: L_B^T x = y - E_r'^T x_f).  The last `band`
// values of each sweep stay in a register shift register.  Two lanes walk the
// cell (half = 0 for lane c, 1 for lane c + 32): of each pair of a step's
// factor values, half 0 loads the first and half 1 the second, and a lane
// swap at compute time gives both lanes both values, so both compute the
// same recurrence and half 0 alone writes the result (half 1 writes the
// scratch slot).  BM >= band, and band >= 2 (the tridiagonal band runs
// wave-per-cell).  Every load address is valid and computed without
// conditions on the step: an absent coefficient (j > band, coupling without
// `arrow`) reads some other factor entry of the cell and is zeroed by a 0/1
// weight in the arithmetic, and a step past the last level reads the last
// level's entries.
template <bool TRANS, int BM, typename T, typename TA>
__device__ __forceinline__ void band_solve_pipe(const T* __restrict__ fb, int L, int m, int band,
                                                int arrow, int half, const T (&s3i)[9],
                                                double* v) {
  // values of a step: the BM band coefficients, the 3 coupling entries and,
  // in the sweep that divides, 1 / u_kk; NP loads of two values each
  constexpr int NP = (BM + 5) / 2;
  constexpr int U = NP <= 3 ? 16 : NP <= 4 ? 15 : 10;  // (U - 1) x NP <= 56
  const int RB = 2 * band + 1 + (arrow ? 6 : 0);        // rows per level
  auto ld = [&](int row, int k) -> T { return fb[((long long)k * RB + row) * BT]; };
  // (row, level) of value q of forward step kk / backward step kk
  auto fwd_at = [&](int q, int kk, int& row, int& lev) {
    const int j = q + 1, i = q - BM;
    if (q < BM) {
      row = TRANS ? (j <= band ? band + j : j - band) : (j <= band ? j - 1 : j - 1 - band);
      lev = TRANS ? max(kk - j, 0) : kk;
    } else if (q < BM + 3) {
      row = arrow ? 2 * band + (TRANS ? 1 : 4) + i : i;
      lev = kk;
    } else {  // 1 / u_kk (TRANS), or an unused value
      row = band;
      lev = kk;
    }
  };
  auto bwd_at = [&](int q, int kk, int& row, int& lev) {
    const int j = q + 1, i = q - BM;
    if (q < BM) {
      row = TRANS ? (j <= band ? j - 1 : j - 1 - band) : (j <= band ? band + j : j - band);
      lev = TRANS ? min(kk + j, L - 1) : kk;
    } else if (q < BM + 3) {
      row = arrow ? 2 * band + (TRANS ? 4 : 1) + i : i;
      lev = kk;
    } else {  // 1 / u_kk (not TRANS), or an unused value
      row = band;
      lev = kk;
    }
  };
  struct Step {
    T raw[NP];  // this lane's half of the step's values
    TA v;       // right-hand side (forward) or the forward result (backward)
  };
  // both lanes of the cell get value 2p (loaded by half 0) in val[2p] and
  // value 2p + 1 (half 1) in val[2p + 1]
  auto unpack = [&](const Step& s, TA (&val)[2 * NP]) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      TA x = (TA)s.raw[p], y = x;
      swap32(x, y);
      val[2 * p] = x;
      val[2 * p + 1] = y;
    }
  };
  TA wj[BM];  // 1 for the band's diagonals, 0 past `band`
#pragma unroll
  for (int j = 0; j < BM; ++j) wj[j] = j < band ? TA(1) : TA(0);
  const TA we = arrow ? TA(1) : TA(0);
  const int sink = m;  // half 1's writes
  TA h[BM];
  TA acc[3] = {TA(0), TA(0), TA(0)};
#pragma unroll
  for (int j = 0; j < BM; ++j) h[j] = TA(0);
  // forward: L_B y = r (TRANS: U_B^T y = r); h[j-1] = y_{k-j}
  ring_walk<U, Step>(
      L,
      [&](int k, Step& s) {
        const int kk = min(k, L - 1);
        s.v = (TA)v[kk];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          int ra, la, rb, lb;
          fwd_at(2 * p, kk, ra, la);
          fwd_at(2 * p + 1, kk, rb, lb);
          s.raw[p] = ld(half ? rb : ra, half ? lb : la);
        }
      },
      [&](int k, const Step& s) {
        TA val[2 * NP];
        unpack(s, val);
        TA y = s.v;
#pragma unroll
        for (int j = BM; j >= 1; --j) y -= (val[j - 1] * wj[j - 1]) * h[j - 1];
        if (TRANS) y *= val[BM + 3];
#pragma unroll
        for (int j = BM - 1; j > 0; --j) h[j] = h[j - 1];
        h[0] = y;
        v[half ? sink : k] = (double)y;
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] += (val[BM + i] * we) * y;
      });
  TA yf[3], xf[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) yf[i] = (TA)v[L + i] - acc[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    xf[i] = (TA)s3i[TRANS ? i : 3 * i] * yf[0] + (TA)s3i[TRANS ? 3 + i : 3 * i + 1] * yf[1] +
            (TA)s3i[TRANS ? 6 + i : 3 * i + 2] * yf[2];
  // backward: U_B x = y - E_c' x_f (TRANS: L_B^T x = y - E_r'^T x_f);
  // h[j-1] = x_{k+j}; step t walks k = L - 1 - t
#pragma unroll
  for (int j = 0; j < BM; ++j) h[j] = TA(0);
  ring_walk<U, Step>(
      L,
      [&](int t, Step& s) {
        const int kk = max(L - 1 - t, 0);
        s.v = (TA)v[kk];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          int ra, la, rb, lb;
          bwd_at(2 * p, kk, ra, la);
          bwd_at(2 * p + 1, kk, rb, lb);
          s.raw[p] = ld(half ? rb : ra, half ? lb : la);
        }
      },
      [&](int t, const Step& s) {
        TA val[2 * NP];
        unpack(s, val);
        TA x = s.v;
#pragma unroll
        for (int i = 0; i < 3; ++i) x -= (val[BM + i] * we) * xf[i];
#pragma unroll
        for (int j = BM; j >= 1; --j) x -= (val[j - 1] * wj[j - 1]) * h[j - 1];
        if (!TRANS) x *= val[BM + 3];
#pragma unroll
        for (int j = BM - 1; j > 0; --j) h[j] = h[j - 1];
        h[0] = x;
        v[half ? sink : L - 1 - t] = (double)x;
      });
#pragma unroll
  for (int i = 0; i < 3; ++i) v[half ? sink : L + i] = (double)xf[i];
}

// The tile's right-hand sides between HBM (row cc of the tile at cc * cs)
// and LDS (row cc at cc * ls), both ways as one flat range of cells x m
// elements: element i is row i / m, column i % m, and each of the
// workgroup's WAVE threads takes every WAVE-th one.  A batch issues all of its loads before any of its writes, so
// that the loads of a batch are in flight together (a row at a time, each
// load would wait for the one before).  i / m comes from a float product
// and one correction each way: i < 2^24, so the product is within one of
// the quotient.
constexpr int STAGE_BATCH = 16;

__device__ __forceinline__ void stage_split(int i, int m, float rm, int& q, int& k) {
  q = (int)((float)i * rm);
  q -= q * m > i ? 1 : 0;
  q += (q + 1) * m <= i ? 1 : 0;
  k = i - q * m;
}

__device__ __forceinline__ void stage_in(const double* __restrict__ src, long long cs, int cells,
                                         int m, double* sv, int ls, int lane) {
  const int tot = cells * m;
  const float rm = 1.0f / (float)m;
  for (int b = 0; b < tot; b += STAGE_BATCH * WAVE) {
    double t[STAGE_BATCH];
    int o[STAGE_BATCH];
#pragma unroll
    for (int u = 0; u < STAGE_BATCH; ++u) {
      const int i = b + u * WAVE + lane;
      int q, k;
      stage_split(min(i, tot - 1), m, rm, q, k);
      t[u] = src[(long long)q * cs + k];
      o[u] = i < tot ? q * ls + k : -1;
    }
#pragma unroll
    for (int u = 0; u < STAGE_BATCH; ++u)
      if (o[u] >= 0) sv[o[u]] = t[u];
  }
}

__device__ __forceinline__ void stage_out(const double* sv, int ls, int cells, int m,
                                          double* __restrict__ dst, long long cs, int lane) {
  const int tot = cells * m;
  const float rm = 1.0f / (float)m;
  for (int b = 0; b < tot; b += STAGE_BATCH * WAVE) {
    double t[STAGE_BATCH];
    long long o[STAGE_BATCH];
#pragma unroll
    for (int u = 0; u < STAGE_BATCH; ++u) {
      const int i = b + u * WAVE + lane;
      int q, k;
      stage_split(min(i, tot - 1), m, rm, q, k);
      t[u] = sv[q * ls + k];
      o[u] = i < tot ? (long long)q * cs + k : -1;
    }
#pragma unroll
    for (int u = 0; u < STAGE_BATCH; ++u)
      if (o[u] >= 0) dst[o[u]] = t[u];
  }
}

// x0 = A0^{-1} r for every right-hand side, two lanes per cell (BT cells per
// wavefront).  The tile's right-hand sides go through LDS ([BT][(m + 1) | 1]:
// an odd row stride, so that the cells' rows fall in different banks, and a
// scratch slot at m), staged in and out as one flat range of elements
// (stage_in, stage_out), while the walk reads and writes its cell's row in
// place.  Lanes past the last cell walk whatever their LDS row holds and
// store nothing.
template <typename TV, bool TRANS, int BM>
__global__ __launch_bounds__(WAVE) void k_band_solve(Mesh g, const TV* __restrict__ bf,
                                                     const TV* __restrict__ s3i_in,
                                                     const double* rin, double* zout, int nrhs,
                                                     long long cs, long long rs) {
  extern __shared__ double sv[];
  const int tile = blockIdx.x, lane = threadIdx.x % BT, half = threadIdx.x / BT;
  const int L = g.L, m = g.m, ls = (m + 1) | 1;
  const long long c0 = (long long)tile * BT;
  const int cells = (int)(g.N - c0 < BT ? g.N - c0 : BT);
  const TV* fb = bf + (long long)tile * band_rows(g) * L * BT + lane;
  double* mine = sv + lane * ls;
  const int r = blockIdx.y;  // one right-hand side per workgroup
  const double* rr = rin + (long long)r * rs + c0 * cs;
  stage_in(rr, cs, cells, m, sv, ls, threadIdx.x);
  __syncthreads();
  // loaded after the barrier (which waits for every load before it), in
  // flight with the walk's first factor loads; first used between the sweeps
  TV s3i[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) s3i[t] = s3i_in[((long long)tile * 9 + t) * BT + lane];
  band_solve_pipe<TRANS, BM, TV, TV>(fb, L, m, g.band, g.arrow, half, s3i, mine);
  __syncthreads();
  double* zz = zout + (long long)r * rs + c0 * cs;
  stage_out(sv, ls, cells, m, zz, cs, threadIdx.x);
}

template <typename TV, bool TRANS, int BM>
static void launch_band_solve(const Mesh& g, const TV* bf, const TV* s3i, const double* r,
                              double* z, int nrhs, hipStream_t s, long long cs = -1,
                              long long rs = -1) {
  if (cs < 0) cs = g.m;  // the [nrhs][N][m] vector layout by default
  if (rs < 0) rs = g.n;
  const size_t lds = (size_t)BT * ((g.m + 1) | 1) * sizeof(double);
  if (lds > 65536)  // up to the 160 KiB of a CU
    (void)hipFuncSetAttribute((const void*)k_band_solve<TV, TRANS, BM>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_band_solve<TV, TRANS, BM>), dim3((unsigned)band_tiles(g), nrhs),
                     dim3(WAVE), lds, s, g, bf, s3i, r, z, nrhs, cs, rs);
}

static void launch_band_cinv(const Mesh& g, const double* wv, double* cinv, int* status,
                             hipStream_t s) {
  const dim3 grid((g.N + WPB - 1) / WPB), block(64 * WPB);
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: hipLaunchKernelGGL(k_band_cinv<1>, grid, block, 0, s, g, wv, cinv, status); break;
    case 2: hipLaunchKernelGGL(k_band_cinv<2>, grid, block, 0, s, g, wv, cinv, status); break;
    case 3: hipLaunchKernelGGL(k_band_cinv<3>, grid, block, 0, s, g, wv, cinv, status); break;
    default: hipLaunchKernelGGL(k_band_cinv<4>, grid, block, 0, s, g, wv, cinv, status); break;
  }
}

// Setup of the banded block-Jacobi: the factorisation (one lane per cell),
// then the Woodbury factors with coalesced, wave-per-cell kernels and the
// apply's pipelined walk: the u / v rows into wv (and wvT), W_i = A0^{-1} u_i
// (A0^{-T} v_i) solved in place as rd right-hand sides of stride mp in
// cell-major rows, then C^{-1}.
hipError_t launch_band_setup(const Mesh& g, const double* rec, double* bf, double* s3i,
                             double* wv, double* wvT, double* cinv, int* status, hipStream_t s) {
  if (g.rd > RANK_DIAG_MAX || g.band > BAND_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_band_setup, dim3((unsigned)band_tiles(g)), dim3(BT), 0, s, g, rec, bf, s3i,
                     status);
  const int cg = (g.N + WPB - 1) / WPB;
  hipLaunchKernelGGL(k_band_wv_init, dim3(cg), dim3(64 * WPB), 0, s, g, rec, wv, wvT);
  const int rd = smw_pairs(g);
  const long long cs = 2LL * rd * g.mp;
  auto solve = [&](auto trans_tag, double* w) {
    constexpr bool TR = decltype(trans_tag)::value;
    if (g.band <= 2)
      launch_band_solve<double, TR, 2>(g, bf, s3i, w, w, rd, s, cs, g.mp);
    else if (g.band <= 4)
      launch_band_solve<double, TR, 4>(g, bf, s3i, w, w, rd, s, cs, g.mp);
    else
      launch_band_solve<double, TR, BAND_MAX>(g, bf, s3i, w, w, rd, s, cs, g.mp);
  };
  solve(std::false_type{}, wv);
  if (wvT) solve(std::true_type{}, wvT);
  launch_band_cinv(g, wv, cinv, status, s);
  return hipGetLastError();
}

// z = x0 - W C^{-1} (V^T x0) in place, one wavefront per cell (NCH chunks of
// 64 unknowns), W and V rows [N][2 rd][mp] of the direction being applied.
template <typename TV, int NCH, bool TRANS, int RDM>
__global__ __launch_bounds__(64 * WPB) void k_band_woodbury(Mesh g, const TV* __restrict__ wv,
                                                            const TV* __restrict__ cinv,
                                                            double* __restrict__ z, int nrhs) {
  const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + (threadIdx.x >> 6)));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m, rd = RDM == 1 ? 1 : smw_pairs(g);
  const long long mp = g.mp;
  const TV* wc = wv + (long long)c * 2 * rd * mp;
  CapInv<TV, RDM> IC;
  IC.load(cinv, c, rd, lane);
  TV W[RDM][NCH], V[RDM][NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const int kk = k < m ? k : m - 1;
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      W[i][ch] = i < rd ? ld_stream(wc + i * mp + kk) : TV(0);
      V[i][ch] = i < rd ? ld_stream(wc + (rd + i) * mp + kk) : TV(0);
    }
  }
  for (int r = 0; r < nrhs; ++r) {
    double* zc = z + (long long)r * g.n + (long long)c * m;
    TV X[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      X[ch] = (TV)zc[k < m ? k : m - 1];
    }
    TV s[RDM], zz[RDM];
#pragma unroll
    for (int g0 = 0; g0 < RDM; g0 += 4) {  // wave sums four at a time
      TV s4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s4[e] = TV(0);
        if (g0 + e < RDM) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            if (ch * WAVE + lane < m) s4[e] += V[g0 + e][ch] * X[ch];
        }
      }
      wave_sums_u(s4);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (g0 + e < RDM) s[g0 + e] = g0 + e < rd ? s4[e] : TV(0);
    }
    IC.template apply<TRANS>(s, zz, rd);
    // every lane has read its entries before any lane writes (the reads
    // above feed the wave sums), so the in-place update is safe
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int k = ch * WAVE + lane;
      TV o = X[ch];
#pragma unroll
      for (int i = 0; i < RDM; ++i) o -= zz[i] * W[i][ch];
      if (k < m) zc[k] = (double)o;
    }
  }
}

template <typename TV, bool TRANS, int RDM>
static void launch_woodbury_r(const Mesh& g, const TV* wv, const TV* cinv, double* z, int nrhs,
                              hipStream_t s) {
  const dim3 grid((g.N + WPB - 1) / WPB), block(64 * WPB);
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: hipLaunchKernelGGL((k_band_woodbury<TV, 1, TRANS, RDM>), grid, block, 0, s, g, wv, cinv, z, nrhs); break;
    case 2: hipLaunchKernelGGL((k_band_woodbury<TV, 2, TRANS, RDM>), grid, block, 0, s, g, wv, cinv, z, nrhs); break;
    case 3: hipLaunchKernelGGL((k_band_woodbury<TV, 3, TRANS, RDM>), grid, block, 0, s, g, wv, cinv, z, nrhs); break;
    default: hipLaunchKernelGGL((k_band_woodbury<TV, 4, TRANS, RDM>), grid, block, 0, s, g, wv, cinv, z, nrhs); break;
  }
}

template <typename TV, bool TRANS>
static hipError_t launch_band_apply_t(const Mesh& g, const TV* bf, const TV* s3i, const TV* wv,
                                      const TV* cinv, const double* r, double* z, int nrhs,
                                      hipStream_t s) {
  if (g.band <= 2)
    launch_band_solve<TV, TRANS, 2>(g, bf, s3i, r, z, nrhs, s);
  else if (g.band <= 4)
    launch_band_solve<TV, TRANS, 4>(g, bf, s3i, r, z, nrhs, s);
  else
    launch_band_solve<TV, TRANS, BAND_MAX>(g, bf, s3i, r, z, nrhs, s);
  const int pw = smw_pairs(g);
  if (pw == 1)
    launch_woodbury_r<TV, TRANS, 1>(g, wv, cinv, z, nrhs, s);
  else if (pw <= RANK_DIAG_MAX)
    launch_woodbury_r<TV, TRANS, RANK_DIAG_MAX>(g, wv, cinv, z, nrhs, s);
  else
    launch_woodbury_r<TV, TRANS, SMW_PAIRS_MAX>(g, wv, cinv, z, nrhs, s);
  return hipGetLastError();
}

hipError_t launch_band_apply(const Mesh& g, const void* bf, const void* s3i, const void* wv,
                             const void* cinv, bool f32, bool trans, const double* r, double* z,
                             int nrhs, hipStream_t s) {
  if (g.rd > RANK_DIAG_MAX || g.band > BAND_MAX || g.m > WAVE * MAX_CHUNKS)
    return hipErrorInvalidValue;
  if (f32)
    return trans ? launch_band_apply_t<float, true>(g, (const float*)bf, (const float*)s3i,
                                                    (const float*)wv, (const float*)cinv, r, z, nrhs, s)
                 : launch_band_apply_t<float, false>(g, (const float*)bf, (const float*)s3i,
                                                     (const float*)wv, (const float*)cinv, r, z, nrhs, s);
  return trans ? launch_band_apply_t<double, true>(g, (const double*)bf, (const double*)s3i,
                                                   (const double*)wv, (const double*)cinv, r, z, nrhs, s)
               : launch_band_apply_t<double, false>(g, (const double*)bf, (const double*)s3i,
                                                    (const double*)wv, (const double*)cinv, r, z, nrhs, s);
}

// ------------------------------------------------------ general pattern ----
// LU without pivoting of B = P S_cc P^T (P the plan's minimum-degree order)
// with the fill the host found, one lane per cell: the factor of cell c is
// nnzF values at positions p of the filled pattern, tile-interleaved
// [tile][p][TILE] like the band factors, with 1 / U[k][k] at the diagonal
// positions.  The solves walk the position tables (wave-uniform, the same
// for every lane) and keep the lane's vector in its original order: the
// value of new index i lives at perm[i] throughout, so that no permutation
// pass is needed.

// x = A0^{-1} v (A0^{-T} v with the transposed stream) in place in v[0 ..
// m): the plan's flat operation stream (forward L y = P v, backward U (P x)
// = y; transposed U^T z = P v, then L^T (P x) = z), each operation one
// factor value times one element of v.  The factor loads of the next U
// operations are issued before the current U are computed (the operations
// themselves are wave-uniform scalar loads); operations past the end are
// dead.  F points at this lane's factor values (stride TILE).  With SINK
// every operation reads and writes v (branch-free: a read that is not needed
// and a write that is not wanted go to the sink element v[m], so the
// operations of a block are straight-line code); without, v needs only m
// elements.
template <int U, bool SINK, typename TA, typename T>
__device__ __forceinline__ void pattern_stream(const int* __restrict__ ops, int nops, int m,
                                               const T* __restrict__ F, double* v) {
  struct Op {
    TA f;
    int code;  // kind << 16 | index, bit 20 set where the END scales by f
  };
  TA acc = TA(0);
  // a block's (pos, code) pairs are read as one contiguous run before any of
  // its factor loads, so that one wait covers the block's scalar loads.  The
  // tables are padded to 256-byte pieces (32 operations), so a block of U <=
  // 32 operations that starts before the end lies inside its piece; blocks
  // past the end reread the last one, and operations past the end are dead.
  static_assert(32 % U == 0, "a block lies inside one 32-operation piece");
  const int last = ((nops - 1) / U) * U;
  pipelined_walk<U, Op>(
      nops,
      [&](int b, Op(&S)[U]) {
        const int2* blk = reinterpret_cast<const int2*>(ops) + min(b * U, last);
        int pos[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int2 pc = blk[u];
          pos[u] = pc.x;
          S[u].code = b * U + u < nops ? pc.y | (pc.x >= 0 ? 1 << 20 : 0) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) S[u].f = (TA)F[(long long)(pos[u] >= 0 ? pos[u] : 0) * TILE];
      },
      [&](int, const Op& o) {
        const int kind = (o.code >> 16) & 15, idx = o.code & 0xffff;
        const bool scale = (o.code >> 20) & 1;
        if constexpr (SINK) {
          const bool upd = kind == PAT_OP_UPD, start = kind == PAT_OP_START;
          const bool end = kind == PAT_OP_END;
          const TA val = (TA)v[upd || start ? idx : m];
          acc = start ? val : acc - (upd ? o.f : TA(0)) * val;
          v[end ? idx : m] = (double)(scale ? acc * o.f : acc);
        } else {
          if (o.code < 0) return;
          if (kind == PAT_OP_UPD)
            acc -= o.f * (TA)v[idx];
          else if (kind == PAT_OP_START)
            acc = (TA)v[idx];
          else
            v[idx] = (double)(scale ? acc * o.f : acc);
        }
      });
}

// One lane per cell: the numeric LU (right-looking: for pivot k, scale
// column k of L, then update the trailing entries (i, j) of row i of L's
// column k and column j of U's row k), then the Woodbury factors.
__global__ __launch_bounds__(TILE) void k_pattern_setup(Mesh g, PatLU lu,
                                                        const double* __restrict__ rec,
                                                        double* __restrict__ bf, int* status) {
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int c = tile * TILE + lane;
  if (c >= g.N) return;  // no cross-lane work in this kernel
  const int m = g.m;
  const long long mp = g.mp;
  const double* rc = rec + (long long)c * g.F * mp;
  double* F = bf + (long long)tile * lu.nnzF * TILE + lane;
  auto at = [&](int p) -> double& { return F[(long long)p * TILE]; };
  for (int p = 0; p < lu.nnzF; ++p) {
    const int o = lu.frec[p];
    at(p) = o >= 0 ? rc[o] : 0.0;
  }
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    const double piv = at(lu.dpos[k]);
    if (!(fabs(piv) > 1e-14 * fabs(rc[F_DIAG * mp + lu.perm[k]]))) bad = true;
    const double inv = 1.0 / piv;
    at(lu.dpos[k]) = inv;
    for (int a = lu.lcol_ptr[k]; a < lu.lcol_ptr[k + 1]; ++a) {
      const double l = at(lu.lcol_pos[a]) * inv;
      at(lu.lcol_pos[a]) = l;
      const int i = lu.lcol_row[a];
      for (int b = lu.urow_ptr[k]; b < lu.urow_ptr[k + 1]; ++b)
        at(lu.posF[i * m + lu.urow_col[b]]) -= l * at(lu.urow_pos[b]);
    }
  }
  if (bad) atomicMin(status, c);
}

// x0 = A0^{-1} r for every right-hand side, one lane per cell, the tile's
// right-hand sides staged through LDS as in k_band_solve.
#ifndef PAT_STREAM_U
// operations per prefetch block (the two blocks' codes fit in scalar
// registers: 94 SGPRs, no spills)
#define PAT_STREAM_U 16
#endif
template <typename TV, bool TRANS>
__global__ __launch_bounds__(TILE) void k_pattern_solve(Mesh g, PatLU lu,
                                                        const TV* __restrict__ bf,
                                                        const double* rin, double* zout,
                                                        long long cs, long long rs) {
  extern __shared__ double sv[];
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int m = g.m, ls = (m + 1) | 1;
  const long long c0 = (long long)tile * TILE;
  const int cells = (int)(g.N - c0 < TILE ? g.N - c0 : TILE);
  const TV* F = bf + (long long)tile * lu.nnzF * TILE + lane;
  double* mine = sv + lane * ls;
  const int r = blockIdx.y;  // one right-hand side per workgroup
  const double* rr = rin + (long long)r * rs + c0 * cs;
  stage_in(rr, cs, cells, m, sv, ls, lane);
  __syncthreads();
  if (TRANS)
    pattern_stream<PAT_STREAM_U, true, TV>(lu.ops_t, lu.nops_t, m, F, mine);
  else
    pattern_stream<PAT_STREAM_U, true, TV>(lu.ops_n, lu.nops_n, m, F, mine);
  __syncthreads();
  double* zz = zout + (long long)r * rs + c0 * cs;
  stage_out(sv, ls, cells, m, zz, cs, lane);
}

template <typename TV, bool TRANS>
static void launch_pattern_solve(const Mesh& g, const PatLU& lu, const TV* bf, const double* r,
                                 double* z, int nrhs, hipStream_t s, long long cs = -1,
                                 long long rs = -1) {
  if (cs < 0) cs = g.m;  // the [nrhs][N][m] vector layout by default
  if (rs < 0) rs = g.n;
  const size_t lds = (size_t)TILE * ((g.m + 1) | 1) * sizeof(double);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_pattern_solve<TV, TRANS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_pattern_solve<TV, TRANS>), dim3((unsigned)tiles(g), nrhs), dim3(TILE), lds,
                     s, g, lu, bf, r, z, cs, rs);
}

// Setup of the general-pattern block-Jacobi: the numeric LU (one lane per
// cell), then the Woodbury factors as for the band (u / v rows, W solved in
// place by the apply's stream walk, C^{-1} wave per cell).
hipError_t launch_pattern_setup(const Mesh& g, const PatLU& lu, const double* rec, double* bf,
                                double* wv, double* wvT, double* cinv, int* status,
                                hipStream_t s) {
  if (!g.pat || g.rd > RANK_DIAG_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pattern_setup, dim3((unsigned)tiles(g)), dim3(TILE), 0, s, g, lu, rec, bf,
                     status);
  const int cg = (g.N + WPB - 1) / WPB;
  hipLaunchKernelGGL(k_band_wv_init, dim3(cg), dim3(64 * WPB), 0, s, g, rec, wv, wvT);
  const int rd = smw_pairs(g);
  const long long cs = 2LL * rd * g.mp;
  launch_pattern_solve<double, false>(g, lu, bf, wv, wv, rd, s, cs, g.mp);
  if (wvT) launch_pattern_solve<double, true>(g, lu, bf, wvT, wvT, rd, s, cs, g.mp);
  launch_band_cinv(g, wv, cinv, status, s);
  return hipGetLastError();
}

template <typename TV, bool TRANS>
static hipError_t launch_pattern_apply_t(const Mesh& g, const PatLU& lu, const TV* bf,
                                         const TV* wv, const TV* cinv, const double* r, double* z,
                                         int nrhs, hipStream_t s) {
  launch_pattern_solve<TV, TRANS>(g, lu, bf, r, z, nrhs, s);
  if (g.rd == 1)
    launch_woodbury_r<TV, TRANS, 1>(g, wv, cinv, z, nrhs, s);
  else
    launch_woodbury_r<TV, TRANS, RANK_DIAG_MAX>(g, wv, cinv, z, nrhs, s);
  return hipGetLastError();
}

hipError_t launch_pattern_apply(const Mesh& g, const PatLU& lu, const void* bf, const void* wv,
                                const void* cinv, bool f32, bool trans, const double* r,
                                double* z, int nrhs, hipStream_t s) {
  if (!g.pat || g.rd > RANK_DIAG_MAX || g.m > WAVE * MAX_CHUNKS) return hipErrorInvalidValue;
  if (f32)
    return trans ? launch_pattern_apply_t<float, true>(g, lu, (const float*)bf, (const float*)wv,
                                                       (const float*)cinv, r, z, nrhs, s)
                 : launch_pattern_apply_t<float, false>(g, lu, (const float*)bf, (const float*)wv,
                                                        (const float*)cinv, r, z, nrhs, s);
  return trans ? launch_pattern_apply_t<double, true>(g, lu, (const double*)bf, (const double*)wv,
                                                      (const double*)cinv, r, z, nrhs, s)
               : launch_pattern_apply_t<double, false>(g, lu, (const double*)bf, (const double*)wv,
                                                       (const double*)cinv, r, z, nrhs, s);
}

void pattern_prec_counts(const Mesh& g, int nnzF, long long* bf, long long* wv, long long* cinv) {
  *bf = tiles(g) * (long long)nnzF * TILE;
  *wv = (long long)g.N * 2 * g.rd * g.mp;
  *cinv = (long long)g.N * g.rd * g.rd;
}

// Element counts of the factor arrays (host layout helper): band factors and
// Schur inverses tile-interleaved, W / V rows and C^{-1} per cell.
void band_prec_counts(const Mesh& g, long long* bf, long long* s3i, long long* wv,
                      long long* cinv) {
  const long long T = band_tiles(g);
  *bf = T * band_rows(g) * g.L * BT;
  *s3i = T * 9 * BT;
  *wv = (long long)g.N * 2 * smw_pairs(g) * g.mp;
  *cinv = (long long)g.N * smw_pairs(g) * smw_pairs(g);
}

}  // namespace r1s
