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
// A band solve is a serial recurrence of order `band`, so here one lane owns
// one cell and walks its levels (64 cells per wavefront) instead of one wave
// per cell with lane-parallel scans: the scan of an order-h recurrence costs
// O(h^3 log 64) per lane, the serial walk O(h) per level.  All factors are
// stored tile-interleaved, [tile of 64 cells][row][k][lane], so the 64 lanes
// of a wave read one factor entry of 64 consecutive cells as one contiguous
// 512-byte run.  Right-hand sides and results keep the [nrhs][N][m] vector
// layout (each lane streams its own cell's contiguous block).
#include <math.h>

#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

constexpr int TILE = 64;

// Row offsets of the band factors inside one tile ([rows][L][64]):
//   lo(j) rows 0..band-1       l_{k,j} = L_B[k][k-j]      (k >= j)
//   ui     row band            1 / U_B[k][k]
//   up(j) rows band+1..2 band  U_B[k][k+j]                 (k + j < L)
//   ec(i) rows 2 band+1+i      (L_B^{-1} E_c)[k][i]        (coupling only)
//   er(i) rows 2 band+4+i      (E_r U_B^{-1})[i][k]        (coupling only)
template <typename T>
struct BandView {
  const T* base;   // this lane's tile, lane offset applied
  int L, band, arrow;
  __device__ inline T at(int row, int k) const { return base[((long long)row * L + k) * TILE]; }
  __device__ inline T lo(int j, int k) const { return at(j - 1, k); }
  __device__ inline T ui(int k) const { return at(band, k); }
  __device__ inline T up(int j, int k) const { return at(band + j, k); }
  __device__ inline T ec(int i, int k) const { return at(2 * band + 1 + i, k); }
  __device__ inline T er(int i, int k) const { return at(2 * band + 4 + i, k); }
};

__host__ __device__ inline int band_rows(const Mesh& g) { return 2 * g.band + 1 + 6 * g.arrow; }
__host__ __device__ inline long long tiles(const Mesh& g) { return (g.N + TILE - 1) / TILE; }

// Solve A0 x = r (TRANS: A0^T x = r) for one cell.  r(k) gives the right-hand
// side; x is written to dst[k * ds] (k < m) and also serves as the scratch of
// the forward sweep.  s3i: the 3 x 3 inverse of the Schur complement (row
// major).  Returns nothing; accumulation in TA.
template <bool TRANS, typename T, typename TA, typename RHS, typename DST>
__device__ inline void band_solve(const BandView<T>& f, const T (&s3i)[9], RHS r, DST* dst,
                                  int ds) {
  const int L = f.L, band = f.band;
  TA acc[3] = {TA(0), TA(0), TA(0)};
  // forward sweep: L_B y = r (TRANS: U_B^T y = r), coupling sums on the way
  for (int k = 0; k < L; ++k) {
    TA y = (TA)r(k);
    for (int j = 1; j <= band && j <= k; ++j)
      y -= (TA)(TRANS ? f.up(j, k - j) : f.lo(j, k)) * (TA)dst[(k - j) * ds];
    if (TRANS) y *= (TA)f.ui(k);
    dst[k * ds] = (DST)y;
    if (f.arrow)
      for (int i = 0; i < 3; ++i) acc[i] += (TA)(TRANS ? f.ec(i, k) : f.er(i, k)) * y;
  }
  // flow unknowns through the Schur complement (TRANS: its transpose)
  TA yf[3], xf[3];
  for (int i = 0; i < 3; ++i) yf[i] = (TA)r(L + i) - acc[i];
  for (int i = 0; i < 3; ++i)
    xf[i] = (TA)s3i[TRANS ? i : 3 * i] * yf[0] + (TA)s3i[TRANS ? 3 + i : 3 * i + 1] * yf[1] +
            (TA)s3i[TRANS ? 6 + i : 3 * i + 2] * yf[2];
  // backward sweep: U_B x = y - E_c' x_f (TRANS: L_B^T x = y - E_r'^T x_f)
  for (int k = L - 1; k >= 0; --k) {
    TA x = (TA)dst[k * ds];
    if (f.arrow)
      for (int i = 0; i < 3; ++i) x -= (TA)(TRANS ? f.er(i, k) : f.ec(i, k)) * xf[i];
    for (int j = 1; j <= band && k + j < L; ++j)
      x -= (TA)(TRANS ? f.lo(j, k + j) : f.up(j, k)) * (TA)dst[(k + j) * ds];
    if (!TRANS) x *= (TA)f.ui(k);
    dst[k * ds] = (DST)x;
  }
  for (int i = 0; i < 3; ++i) dst[(L + i) * ds] = (DST)xf[i];
}

// ---------------------------------------------------------------- setup ----
// One lane per cell (workgroups of 64 = one tile).  Writes the band factors,
// the Schur inverse (s3i [tile][9][64]), W and V rows for the forward apply
// (wv [tile][2 rd][m][64]: W_i = A0^{-1} u_i, then v_i) and, when wvT is
// given, for the transposed apply (A0^{-T} v_i, then u_i), and C^{-1}
// ([tile][rd^2][64], row-major per cell).
__global__ __launch_bounds__(TILE) void k_band_setup(Mesh g, const double* __restrict__ rec,
                                                     double* __restrict__ bf,
                                                     double* __restrict__ s3i_out,
                                                     double* __restrict__ wv,
                                                     double* __restrict__ wvT,
                                                     double* __restrict__ cinv, int* status) {
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int c = tile * TILE + lane;
  if (c >= g.N) return;  // no cross-lane work in this kernel
  const int L = g.L, m = g.m, band = g.band, rd = g.rd;
  const long long mp = g.mp;
  const double* rc = rec + (long long)c * g.F * mp;
  const int RB = band_rows(g);
  double* fb = bf + (long long)tile * RB * L * TILE + lane;
  auto F = [&](int row, int k) -> double& { return fb[((long long)row * L + k) * TILE]; };
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
  for (int t = 0; t < 9; ++t) s3i_out[((long long)tile * 9 + t) * TILE + lane] = s3i[t];
  for (int k = 0; k < L; ++k) F(band, k) = 1.0 / F(band, k);

  BandView<double> bv{fb, L, band, g.arrow};
  const double* uC = rc + (long long)(g.fu + pair_start(g, D_C)) * mp;
  const double* vC = rc + (long long)(g.fu + g.P + pair_start(g, D_C)) * mp;
  double* wt = wv + (long long)tile * 2 * rd * m * TILE + lane;
  // SMW-1: W_i = A0^{-1} u_i; V_i = v_i
  double vv = 0.0, ww = 0.0;
  for (int i = 0; i < rd; ++i) {
    double* Wi = wt + (long long)i * m * TILE;
    double* Vi = wt + (long long)(rd + i) * m * TILE;
    band_solve<false, double, double>(bv, s3i, [&](int k) { return uC[i * mp + k]; }, Wi, TILE);
    for (int k = 0; k < m; ++k) {
      const double v = vC[i * mp + k];
      Vi[k * TILE] = v;
      vv += v * v;
      ww += Wi[k * TILE] * Wi[k * TILE];
    }
  }
  // SMW-2: C = I + V^T W, inverted by Gauss-Jordan with partial pivoting
  double Cm[RANK_DIAG_MAX][2 * RANK_DIAG_MAX];
  for (int i = 0; i < rd; ++i)
    for (int j = 0; j < rd; ++j) {
      double s = i == j ? 1.0 : 0.0;
      const double* Vi = wt + (long long)(rd + i) * m * TILE;
      const double* Wj = wt + (long long)j * m * TILE;
      for (int k = 0; k < m; ++k) s += Vi[k * TILE] * Wj[k * TILE];
      Cm[i][j] = s;
      Cm[i][rd + j] = i == j ? 1.0 : 0.0;
    }
  const double tol = 1e-12 * (1.0 + sqrt(vv * ww));
  for (int k = 0; k < rd; ++k) {
    int p = k;
    for (int i = k + 1; i < rd; ++i)
      if (fabs(Cm[i][k]) > fabs(Cm[p][k])) p = i;
    if (!(fabs(Cm[p][k]) > tol)) bad = true;
    if (p != k)
      for (int j = 0; j < 2 * rd; ++j) {
        const double t = Cm[k][j];
        Cm[k][j] = Cm[p][j];
        Cm[p][j] = t;
      }
    const double inv = 1.0 / Cm[k][k];
    for (int j = 0; j < 2 * rd; ++j) Cm[k][j] *= inv;
    for (int i = 0; i < rd; ++i) {
      if (i == k) continue;
      const double f = Cm[i][k];
      for (int j = 0; j < 2 * rd; ++j) Cm[i][j] -= f * Cm[k][j];
    }
  }
  double* ci = cinv + (long long)tile * rd * rd * TILE + lane;
  for (int i = 0; i < rd; ++i)
    for (int j = 0; j < rd; ++j) ci[(long long)(i * rd + j) * TILE] = Cm[i][rd + j];
  if (wvT) {  // transposed apply: A0^{-T} v_i and u_i
    double* wtT = wvT + (long long)tile * 2 * rd * m * TILE + lane;
    for (int i = 0; i < rd; ++i) {
      double* Wi = wtT + (long long)i * m * TILE;
      double* Vi = wtT + (long long)(rd + i) * m * TILE;
      band_solve<true, double, double>(bv, s3i, [&](int k) { return vC[i * mp + k]; }, Wi, TILE);
      for (int k = 0; k < m; ++k) Vi[k * TILE] = uC[i * mp + k];
    }
  }
  if (bad) atomicMin(status, c);
}

hipError_t launch_band_setup(const Mesh& g, const double* rec, double* bf, double* s3i,
                             double* wv, double* wvT, double* cinv, int* status, hipStream_t s) {
  if (g.rd > RANK_DIAG_MAX || g.band > BAND_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_band_setup, dim3((unsigned)tiles(g)), dim3(TILE), 0, s, g, rec, bf, s3i, wv,
                     wvT, cinv, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- apply ----
// z = x0 - W C^{-1} (V^T x0), x0 = A0^{-1} r (TRANS: the transposed factors
// and (C^{-1})^T).  One lane per cell; V^T x0 is summed in the backward
// sweep's order of the levels, then the flow unknowns.
template <typename TV, bool TRANS, int RDM>
__global__ __launch_bounds__(TILE) void k_band_apply(Mesh g, const TV* __restrict__ bf,
                                                     const TV* __restrict__ s3i_in,
                                                     const TV* __restrict__ wv,
                                                     const TV* __restrict__ cinv,
                                                     const double* __restrict__ rin,
                                                     double* __restrict__ zout, int nrhs) {
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int c = tile * TILE + lane;
  if (c >= g.N) return;
  const int L = g.L, m = g.m, rd = RDM == 1 ? 1 : g.rd;
  const int RB = band_rows(g);
  BandView<TV> bv{bf + (long long)tile * RB * L * TILE + lane, L, g.band, g.arrow};
  TV s3i[9];
  for (int t = 0; t < 9; ++t) s3i[t] = s3i_in[((long long)tile * 9 + t) * TILE + lane];
  const TV* wt = wv + (long long)tile * 2 * rd * m * TILE + lane;
  const TV* ci = cinv + (long long)tile * rd * rd * TILE + lane;
  for (int r = 0; r < nrhs; ++r) {
    const double* rv = rin + (long long)r * g.n + (long long)c * m;
    double* zv = zout + (long long)r * g.n + (long long)c * m;
    band_solve<TRANS, TV, TV>(bv, s3i, [&](int k) { return rv[k]; }, zv, 1);
    TV s[RDM], z[RDM];
    for (int i = 0; i < RDM; ++i) s[i] = TV(0);
    for (int k = 0; k < m; ++k) {
      const TV xk = (TV)zv[k];
#pragma unroll
      for (int i = 0; i < RDM; ++i)
        if (i < rd) s[i] += wt[((long long)(rd + i) * m + k) * TILE] * xk;
    }
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      TV a = TV(0);
#pragma unroll
      for (int l = 0; l < RDM; ++l)
        if (i < rd && l < rd) a += ci[(long long)(TRANS ? l * rd + i : i * rd + l) * TILE] * s[l];
      z[i] = a;
    }
    for (int k = 0; k < m; ++k) {
      TV o = (TV)zv[k];
#pragma unroll
      for (int i = 0; i < RDM; ++i)
        if (i < rd) o -= z[i] * wt[((long long)i * m + k) * TILE];
      zv[k] = (double)o;
    }
  }
}

template <typename TV, bool TRANS>
static hipError_t launch_band_apply_t(const Mesh& g, const TV* bf, const TV* s3i, const TV* wv,
                                      const TV* cinv, const double* r, double* z, int nrhs,
                                      hipStream_t s) {
  const dim3 grid((unsigned)tiles(g)), block(TILE);
  if (g.rd == 1)
    hipLaunchKernelGGL((k_band_apply<TV, TRANS, 1>), grid, block, 0, s, g, bf, s3i, wv, cinv, r, z, nrhs);
  else
    hipLaunchKernelGGL((k_band_apply<TV, TRANS, RANK_DIAG_MAX>), grid, block, 0, s, g, bf, s3i, wv,
                       cinv, r, z, nrhs);
  return hipGetLastError();
}

hipError_t launch_band_apply(const Mesh& g, const void* bf, const void* s3i, const void* wv,
                             const void* cinv, bool f32, bool trans, const double* r, double* z,
                             int nrhs, hipStream_t s) {
  if (g.rd > RANK_DIAG_MAX || g.band > BAND_MAX) return hipErrorInvalidValue;
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

// Element counts of the tile-interleaved arrays (host layout helper).
void band_prec_counts(const Mesh& g, long long* bf, long long* s3i, long long* wv,
                      long long* cinv) {
  const long long T = tiles(g);
  *bf = T * band_rows(g) * g.L * TILE;
  *s3i = T * 9 * TILE;
  *wv = T * 2 * g.rd * g.m * TILE;
  *cinv = T * g.rd * g.rd * TILE;
}

}  // namespace r1s
