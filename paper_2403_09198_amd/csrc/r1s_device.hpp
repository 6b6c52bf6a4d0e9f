// Device-side helpers shared by the r1s kernels (gfx950, wave64).
//
// Internal layout of the packed Jacobian ("record" layout): one contiguous
// record per mesh cell, [N][F][mp] values, F field rows of mp = m rounded up
// to a multiple of 8 (64-byte rows).  Lane k of the wave that owns cell c
// reads element k of every row, so every load is one contiguous run.
//
//   row 0          diag  S_cc[k][k]
//   row 1          lo    level k: S_cc[k][k-1]; flow row i: S_cc[L+i][L+(i+2)%3]
//   row 2          hi    level k: S_cc[k][k+1]; flow row i: S_cc[L+i][L+(i+1)%3]
//   rows 3..6      nbr   diagonal of S_{c,d}, d = S, W, E, N
//                        (general mesh: rows 3..2+nbmax, one per neighbour slot)
//   fb + j - 2     band  S_cc[k][k-j], j = 2..band (level rows only)
//   fb + band-1 + j-2    S_cc[k][k+j]
//   fa + i         S_cc[k][L+i] (level rows), i < 3, with level/flow coupling
//   fa + 3 + i     S_cc[L+i][k] at index k (the flow row i over the levels)
//   fa + 6         arrow = 2: the atom column S_cc[k][a] at index k < a
//   fa + 7         arrow = 2: the atom row S_cc[a][k] at index k < a
//                  (a = L - 1, the atom density; zero at k >= a)
//   fu .. fu+P-1   u     the pairs of blocks S, W, C, E, N in that order
//                        (ro pairs per neighbour block, rd for the diagonal;
//                        general mesh: the diagonal block's rd, then slot by
//                        slot ro each)
//   fu+P .. F-1    v     same order
// fb = 3 + nbmax (7 on the structured mesh), fa = fb + 2 (band - 1),
// fu = fa + 2 * (coupling slots: 0, 3 or 4), F = fu + 2 P (17 rows with one
// pair per block, band 1 and no coupling).
//
// Padding elements and the rows of blocks that do not exist (mesh boundary)
// are zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace r1s {

constexpr int WAVE = 64;
#ifndef R1S_WPB
#define R1S_WPB 2  // 256 x 128, L = 61: matvec 53.9 us against 54.7 with 4 or 8
#endif
constexpr int WPB = R1S_WPB;
#ifndef R1S_MV_BAND
// Wave-per-cell matvec on column-band tiles (1) or in cell order (0).  256 x
// 128, L = 61, eight right-hand sides: the band map cuts the matvec's fetched
// bytes from 1.64x to 1.02x of its algorithmic reads (the W/E neighbours'
// x blocks no longer go to three XCDs' L2s) but gains only 1% in time; the
// waves wait on memory 64% of their cycles at 5 waves per SIMD.
#define R1S_MV_BAND 1
#endif  // wavefronts (cells) per workgroup of the cell kernels (even)
constexpr int NXCD = 8;      // MI355X: 8 XCDs x 32 CUs
constexpr int F_DIAG = 0, F_LO = 1, F_HI = 2, F_NBR = 3, F_BAND = 7;
// General mesh: neighbour slot s is addressed as direction GSLOT + s.
constexpr int GSLOT = 5, GRAPH_NBR_MAX = 8;
constexpr int D_S = 0, D_W = 1, D_C = 2, D_E = 3, D_N = 4;
constexpr int MAX_CHUNKS = 4;  // m <= 256
// Largest pair counts of the general-rank kernels (a diagonal block / a
// neighbour block); one pair per block has kernels of its own, and up to
// RANK_OFF_SMALL pairs per neighbour block a lighter instantiation.
constexpr int RANK_DIAG_MAX = 9, RANK_OFF_MAX = 6, RANK_OFF_SMALL = 2;
// Woodbury terms of the block-Jacobi at most: the diagonal pairs and the
// atom's column and row
constexpr int SMW_PAIRS_MAX = RANK_DIAG_MAX + 2;
constexpr int BAND_MAX = 8;  // level-band half-width of S_cc
// General pattern of S_cc: at most PAT_ELL_MAX entries per row (and per
// column) outside the dense indices, at most PAT_SLOTS_MAX dense indices
constexpr int PAT_ELL_MAX = 16, PAT_SLOTS_MAX = 8;

// SMW factor records, [N][3 + 2 rd][mp] per direction of application, plus
// the rd x rd inverse capacitance per cell ([N][rd][rd], row-major).
//   forward:   a = -l_k,  dinv = 1/d_k,  b = -s_k/d_k,
//              W_i = S_cc^{-1} u_i, V_i = v_i   (i < rd, the diagonal pairs)
//   transpose: a = -s_{k-1}/d_k, dinv, b = -l_{k+1},
//              W_i = S_cc^{-T} v_i, V_i = u_i, and the transposed C^{-1}
// Flow lanes L+i hold row i of the 3x3 corner inverse (transpose: of its
// transpose) in the a / dinv / b rows.
constexpr int P_A = 0, P_DINV = 1, P_B = 2, P_W = 3;  // V rows at P_W + rd

// Record row length: m values, padded to a multiple of 8 from 64 on.  Below
// 64 the packed kernels read row f of several consecutive cells per load and
// unpadded rows save lines (512 x 256, L = 32, m = 35: matvec 128.6 against
// 135.2 us); from 64 on, 64-byte aligned rows are faster (L = 200, m = 203:
// SMW apply 249.7 against 265.7 us unpadded).
__host__ __device__ inline int pad_m(int m) { return m < 64 ? m : (m + 7) & ~7; }
__host__ __device__ inline int nbr_slot(int d) { return d < 2 ? d : d - 1; }
__host__ __device__ inline int opposite(int d) { return 4 - d; }

struct Mesh {
  int nx, ny, L, m, mp;
  int N;           // nx*ny
  long long n;     // N*m, stride between right-hand sides
  int rd, ro;      // rank-one pairs of a diagonal / a neighbour block
  int P;           // pairs per cell, rd + 4 ro
  int band, arrow; // level-band half-width of S_cc; level/flow coupling
  int fb, fa, fu;  // first band row (j >= 2), first coupling row, first u row
  int F;           // record rows per cell, fu + 2 P
  // general mesh (graph = 1): nbmax neighbour slots per cell; device tables
  // [N][nbmax]: nbr = neighbour cell of each slot (-1: none), tslot = the
  // slot of this cell in the neighbour's list; offb [N] = first off-diagonal
  // block of each cell in input order
  int graph, nbmax;
  const int* nbr;
  const int* tslot;
  const int* offb;
  // general pattern of S_cc (pat = 1): ne ELL rows from fb, ns dense indices
  // px[t] (column row fa + t, row row fa + ns + t); shared tables: pcol
  // [mp][4] the ELL columns of a lane as 16 bytes, ptpos [mp][8] the
  // transposed ELL of a lane as 16 halfwords (slot << 8 | row, 0xffff for
  // none), ppack [1 + ne + 2 ns][mp] entry feeding each record element (-1),
  // perow / pecol / peoff [nnz] the entries' coordinates and record offsets,
  // pdense [m][m] entry at (i, j); ptcol unused
  int pat, ne, net, ns, pnnz;
  int px[PAT_SLOTS_MAX];
  const int *pcol, *ptpos, *ptcol, *ppack, *perow, *pecol, *peoff, *pdense;
};

// Tables of the LU of a general pattern (see pattern.hpp): perm (new ->
// original index), frec (record offset of each factor position, -1 for
// fill), dpos, posF [m][m], strict L and U by rows and by columns.
constexpr int PAT_OP_UPD = 0, PAT_OP_START = 1, PAT_OP_END = 2;
struct PatLU {
  int nnzF, nops_n, nops_t;
  const int *ops_n, *ops_t;  // flat solve streams (see pattern.hpp)
  const int *perm, *frec, *dpos, *posF;
  const int *lrow_ptr, *lrow_pos, *lrow_oc;
  const int *urow_ptr, *urow_pos, *urow_col, *urow_oc;
  const int *lcol_ptr, *lcol_pos, *lcol_row, *lcol_or;
  const int *ucol_ptr, *ucol_pos, *ucol_or;
};

// Band or coupling beyond the tridiagonal / uncoupled diagonal block.
__host__ __device__ inline bool wide_pattern(const Mesh& g) { return g.band > 1 || g.arrow || g.pat; }

// Coupling slots of the diagonal block: slot i < 3 couples the levels to the
// flow unknown L + i; with arrow = 2, slot 3 couples the molecule levels to
// the atom density a = L - 1 (the DRa processes of section 4, "Temporal
// Source Jacobian").  Each slot has a column row (S[k][X_i] at lane k) and a
// row row (S[X_i][k] at lane k) in the record.
constexpr int ARROW_SLOTS_MAX = 4;
__host__ __device__ inline int arrow_slots(const Mesh& g) { return g.arrow == 2 ? 4 : g.arrow ? 3 : 0; }
__host__ __device__ inline int arrow_unknown(int L, int i) { return i < 3 ? L + i : L - 1; }
__host__ __device__ inline int arrow_col_row(const Mesh& g, int i) { return g.fa + (i < 3 ? i : 6); }
__host__ __device__ inline int arrow_row_row(const Mesh& g, int i) { return g.fa + (i < 3 ? 3 + i : 7); }

// First record slot and number of the pairs of block direction d (general
// mesh: d = D_C or GSLOT + slot).
__host__ __device__ inline int pair_count(const Mesh& g, int d) { return d == 2 ? g.rd : g.ro; }
__host__ __device__ inline int pair_start(const Mesh& g, int d) {
  if (g.graph) return d == D_C ? 0 : g.rd + (d - GSLOT) * g.ro;
  return d <= 1 ? d * g.ro : d == 2 ? 2 * g.ro : d == 3 ? 2 * g.ro + g.rd : 3 * g.ro + g.rd;
}
// Record row of the diagonal of the off-diagonal block of direction d.
__host__ __device__ inline int nbr_row(const Mesh& g, int d) {
  return F_NBR + (g.graph ? d - GSLOT : (d < 2 ? d : d - 1));
}
// Woodbury terms of the block-Jacobi: the diagonal block's rd pairs and, with
// arrow = 2, two more for the atom's column and row (u = atom column, v =
// e_a; u = e_a, v = atom row), so that A0 keeps the three-slot pattern.
__host__ __device__ inline int smw_pairs(const Mesh& g) { return g.rd + (g.arrow == 2 ? 2 : 0); }
// Rows of the wave-per-cell SMW factor record of a cell: the three sweep
// rows, W and V (smw_pairs each), and with level/flow coupling the three
// columns T^{-1} E and the three coupling rows of the Schur step.
__host__ __device__ inline int smw_rows(const Mesh& g) { return 3 + 2 * smw_pairs(g) + (g.arrow ? 6 : 0); }
__host__ __device__ inline int smw_arrow_row(const Mesh& g) { return 3 + 2 * smw_pairs(g); }
// The block-Jacobi needs the one-lane-per-cell factorisation when the level
// band is wider than tridiagonal or the pattern is a general one; the
// tridiagonal band, with or without level/flow coupling, runs wave-per-cell.
__host__ __device__ inline bool band_walk(const Mesh& g) { return g.band > 1 || g.pat; }

// Workgroup id -> logical tile.  With R1S_XCD_REMAP each XCD (which
// receives every NXCD-th workgroup) works on one contiguous range of tiles;
// measured on MI355X this is slower for the cell kernels than the hardware's
// round-robin order (all XCDs streaming neighbouring memory), so the default
// keeps the identity map.
__device__ inline int xcd_tile(int bid, int grid) {
#ifndef R1S_XCD_REMAP
  return bid;
#endif
  const int xcd = bid % NXCD, local = bid / NXCD;
  const int per = grid / NXCD, rem = grid % NXCD;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// ------------------------------------------------------------ tile maps ----
// Column-band map: tiles are TQ consecutive cells of one mesh row inside one
// of NXCD column bands, and workgroup b takes band b % NXCD, row by row.
// The dispatcher sends workgroup b to XCD b % NXCD, so each XCD sweeps one
// column band upwards: the x blocks a cell reads from its S, W, E and N
// neighbours were read moments before by the same XCD and come from its L2.
// (Consecutive cells dealt round-robin over the XCDs fetch each x block into
// three L2s, and N/S rows apart again from HBM.)
__host__ __device__ inline int band_tiles(int nx, int TQ) {
  const int bw = (nx + NXCD - 1) / NXCD;
  return (bw + TQ - 1) / TQ;
}
__host__ inline int band_grid(const Mesh& g, int TQ) { return NXCD * g.ny * band_tiles(g.nx, TQ); }

// First cell and cell count (0: an empty tile of a narrow band) of tile b.
__device__ inline void band_tile(const Mesh& g, int b, int TQ, int& c0, int& qn) {
  const int band = b % NXCD, local = b / NXCD;
  const int tb = band_tiles(g.nx, TQ);
  const int iy = local / tb, s = local - iy * tb;
  const int x0 = (int)((long long)band * g.nx / NXCD);
  const int x1 = (int)((long long)(band + 1) * g.nx / NXCD);
  const int a = x0 + s * TQ;
  c0 = iy * g.nx + a;
  const int w = x1 - a;
  qn = iy < g.ny ? (w < TQ ? (w > 0 ? w : 0) : TQ) : 0;
}

// Plain map: tile b is cells b TQ .. b TQ + TQ - 1.
__device__ inline void plain_tile(const Mesh& g, int b, int TQ, int& c0, int& qn) {
  c0 = b * TQ;
  qn = g.N - c0 < TQ ? g.N - c0 : TQ;
}

template <bool BAND>
__device__ inline void cell_tile(const Mesh& g, int b, int TQ, int& c0, int& qn) {
  if (BAND)
    band_tile(g, b, TQ, c0, qn);
  else
    plain_tile(g, b, TQ, c0, qn);
}
template <bool BAND>
__host__ inline int cell_grid(const Mesh& g, int TQ) {
  return BAND ? band_grid(g, TQ) : (g.N + TQ - 1) / TQ;
}

__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }

// Load of streamed matrix data (read once per kernel), marked non-temporal
// so that it does not evict the reused x blocks from L2 (R1S_TEMPORAL builds
// use ordinary loads).
template <typename T>
__device__ inline T ld_stream(const T* p) {
#ifdef R1S_TEMPORAL
  return *p;
#else
  return __builtin_nontemporal_load(p);
#endif
}

// Matrix load of a kernel in which two waves of a workgroup read the same
// record (two halves of a batch of right-hand sides): an ordinary load, so
// that the second wave's read hits L2 instead of refetching from HBM (a
// non-temporal line is not kept for it); else ld_stream.
template <bool SHARED, typename T>
__device__ inline T ld_mat(const T* p) {
  if constexpr (SHARED)
    return *p;
  else
    return ld_stream(p);
}

// Store of a kernel's output vector, non-temporal: an output written back
// through the caches as ordinary lines competes with the streamed matrix
// reads for HBM turnarounds.  Measured on MI355X: a streaming read with 1/16
// as many bytes written drops from 7.37 TB/s to 5.78 with ordinary stores
// and to 5.94 with non-temporal ones; the 512 x 256, L = 200 matvec + SMW
// apply pair takes 934-942 us against 1053 us with ordinary stores.  Even
// where the next kernel reads the output back (the apply after the matvec)
// and an ordinary store would leave it in the Infinity Cache, non-temporal
// stores measured faster (256 x 128, L = 61: 75.6-76.5 us against
// 77.3-79.1 us per pair).
__device__ inline void st_out(double* p, double v) { __builtin_nontemporal_store(v, p); }

// Neighbour cells of c in the order S, W, C, E, N (-1 where no block).
__device__ inline void neighbours(const Mesh& g, int c, int nb[5]) {
  const int iy = c / g.nx, ix = c - iy * g.nx;
  nb[D_S] = iy > 0 ? c - g.nx : -1;
  nb[D_W] = ix > 0 ? c - 1 : -1;
  nb[D_C] = c;
  nb[D_E] = ix < g.nx - 1 ? c + 1 : -1;
  nb[D_N] = iy < g.ny - 1 ? c + g.nx : -1;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Inclusive scan of affine maps y -> a*y + b along increasing lane index:
// on return lane k holds the composition of the maps of lanes 0..k.
template <typename T>
__device__ inline void scan_affine_up(T& a, T& b) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const T ap = __shfl_up(a, off, WAVE);
    const T bp = __shfl_up(b, off, WAVE);
    if (lane >= off) {
      b = a * bp + b;
      a = a * ap;
    }
  }
}

// Same along decreasing lane index (lane k composes lanes 63..k).
template <typename T>
__device__ inline void scan_affine_down(T& a, T& b) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const T ap = __shfl_down(a, off, WAVE);
    const T bp = __shfl_down(b, off, WAVE);
    if (lane + off < WAVE) {
      b = a * bp + b;
      a = a * ap;
    }
  }
}

// ------------------------------------------------ DPP wave primitives ----
// Cross-lane moves in the VALU (data-parallel primitives) instead of LDS
// permutes.  A 64-bit value moves as two 32-bit halves with the same control.
// Rows are groups of 16 lanes; combining the four row results goes through
// v_readlane (wave-uniform values), so no row-broadcast control is needed.
constexpr int DPP_ROW_SHL = 0x100;   // + n: lane l reads lane l + n of its row
constexpr int DPP_ROW_SHR = 0x110;   // + n: lane l reads lane l - n of its row
constexpr int DPP_QP_1032 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int DPP_QP_2301 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

template <int CTRL>
__device__ inline float dpp(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp(double old, double v) {
  const long long o = __double_as_longlong(old), s = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double readlane(double v, int l) {
  const long long s = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)s, l);
  const int hi = __builtin_amdgcn_readlane((int)(s >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, returned wave-uniform.  Fixed association order,
// so the result is bitwise reproducible.
template <typename T>
__device__ inline T wave_sum_u(T v) {
  v += dpp<DPP_QP_1032>(T(0), v);
  v += dpp<DPP_QP_2301>(T(0), v);
  v += dpp<DPP_HALF_MIRROR>(T(0), v);
  v += dpp<DPP_MIRROR>(T(0), v);  // every lane holds its row's sum
  return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}

// Sums over the 64 lanes of K values at once, each returned wave-uniform
// in place.  A reduce-scatter on the gfx950 lane swaps instead of K
// separate reductions: v_permlane32_swap exchanges the upper 32 lanes of one
// register with the lower 32 of another, so one swap and one add fold two
// values over the wave's halves (value 2i in lanes 0-31, 2i+1 in 32-63);
// v_permlane16_swap (odd rows of one register with even rows of the other)
// folds the two resulting registers over row pairs, leaving four values per
// register, one per row; DPP then sums within rows and v_readlane takes each
// row's total.  About a third of the instructions of K wave_sum_u calls
// for K >= 4 (groups of four already reach that rate: callers with many
// sums reduce four at a time, which keeps few partials live).  Every value
// is summed by the same association tree, whatever its position: bitwise
// reproducible, and equal between kernels that group their sums
// differently.
__device__ inline void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ inline void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ inline void swap32(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ inline void swap16(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

template <typename T, int K>
__device__ inline void wave_sums_u(T (&v)[K]) {
  constexpr int K1 = (K + 1) / 2, K2 = (K1 + 1) / 2;
  T h[2 * K2];  // after the first fold: values 2i (lanes 0-31) and 2i + 1 (32-63)
#pragma unroll
  for (int i = 0; i < 2 * K2; ++i) {
    T a = 2 * i < K ? v[2 * i] : T(0);
    T b = 2 * i + 1 < K ? v[2 * i + 1] : T(0);
    if (2 * i < K) {
      swap32(a, b);
      h[i] = a + b;
    } else {
      h[i] = T(0);
    }
  }
  // second fold: register j holds values 4j, 4j + 2, 4j + 1, 4j + 3 in rows
  // 0, 1, 2, 3
  T q[K2];
#pragma unroll
  for (int j = 0; j < K2; ++j) {
    T a = h[2 * j], b = h[2 * j + 1];
    swap16(a, b);
    q[j] = a + b;
  }
#pragma unroll
  for (int j = 0; j < K2; ++j) {
    T x = q[j];
    x += dpp<DPP_QP_1032>(T(0), x);
    x += dpp<DPP_QP_2301>(T(0), x);
    x += dpp<DPP_HALF_MIRROR>(T(0), x);
    x += dpp<DPP_MIRROR>(T(0), x);
    if (4 * j < K) v[4 * j] = readlane(x, 0);
    if (4 * j + 2 < K) v[4 * j + 2] = readlane(x, 16);
    if (4 * j + 1 < K) v[4 * j + 1] = readlane(x, 32);
    if (4 * j + 3 < K) v[4 * j + 3] = readlane(x, 48);
  }
}

// Block and pair of flat index w of a cell's pair coefficients, ordered by
// block (S, W, C, E, N) and pair: RDM pairs for the diagonal block, ROM for
// each neighbour.
template <int RDM, int ROM>
__device__ constexpr void pair_index(int w, int& d, int& p) {
  d = 0;
  for (int dd = 0; dd < 5; ++dd) {
    const int cnt = dd == D_C ? RDM : ROM;
    if (w < cnt) {
      d = dd;
      p = w;
      return;
    }
    w -= cnt;
  }
  p = 0;
}

// Inclusive scan of affine maps y -> a*y + b along increasing lane index
// (lane l ends with the composition of lanes 0..l).  Within rows by DPP
// shifts with the identity map (1, 0) shifted in; then every row is prefixed
// with the composition of the rows below it.
template <typename T>
__device__ inline void scan_affine_up_dpp(T& a, T& b) {
#define R1S_SCAN_STEP(N)                        \
  {                                             \
    const T ap = dpp<DPP_ROW_SHR + N>(T(1), a); \
    const T bp = dpp<DPP_ROW_SHR + N>(T(0), b); \
    b = a * bp + b;                             \
    a = a * ap;                                 \
  }
  R1S_SCAN_STEP(1) R1S_SCAN_STEP(2) R1S_SCAN_STEP(4) R1S_SCAN_STEP(8)
#undef R1S_SCAN_STEP
  const T a0 = readlane(a, 15), b0 = readlane(b, 15);
  const T a1 = readlane(a, 31), b1 = readlane(b, 31);
  const T a2 = readlane(a, 47), b2 = readlane(b, 47);
  // prefixes entering rows 1, 2, 3
  const T pa1 = a0, pb1 = b0;
  const T pa2 = a1 * pa1, pb2 = a1 * pb1 + b1;
  const T pa3 = a2 * pa2, pb3 = a2 * pb2 + b2;
  const int row = lane_id() >> 4;
  const T pa = row == 0 ? T(1) : row == 1 ? pa1 : row == 2 ? pa2 : pa3;
  const T pb = row == 0 ? T(0) : row == 1 ? pb1 : row == 2 ? pb2 : pb3;
  b = a * pb + b;
  a = a * pa;
}

// Same along decreasing lane index (lane l composes lanes 63..l).
template <typename T>
__device__ inline void scan_affine_down_dpp(T& a, T& b) {
#define R1S_SCAN_STEP(N)                        \
  {                                             \
    const T ap = dpp<DPP_ROW_SHL + N>(T(1), a); \
    const T bp = dpp<DPP_ROW_SHL + N>(T(0), b); \
    b = a * bp + b;                             \
    a = a * ap;                                 \
  }
  R1S_SCAN_STEP(1) R1S_SCAN_STEP(2) R1S_SCAN_STEP(4) R1S_SCAN_STEP(8)
#undef R1S_SCAN_STEP
  const T a3 = readlane(a, 48), b3 = readlane(b, 48);
  const T a2 = readlane(a, 32), b2 = readlane(b, 32);
  const T a1 = readlane(a, 16), b1 = readlane(b, 16);
  // suffixes entering rows 2, 1, 0
  const T sa2 = a3, sb2 = b3;
  const T sa1 = a2 * sa2, sb1 = a2 * sb2 + b2;
  const T sa0 = a1 * sa1, sb0 = a1 * sb1 + b1;
  const int row = lane_id() >> 4;
  const T sa = row == 3 ? T(1) : row == 2 ? sa2 : row == 1 ? sa1 : sa0;
  const T sb = row == 3 ? T(0) : row == 2 ? sb2 : row == 1 ? sb1 : sb0;
  b = a * sb + b;
  a = a * sa;
}

// Inclusive scan of 2x2 matrix products along increasing lane index: lane l
// ends with P_l = M_l M_{l-1} ... M_0 (later factors on the left).  Rows of
// 16 lanes by DPP shifts with the identity shifted in, then each row is
// multiplied by the product of the rows below it.
template <typename T>
__device__ inline void mat2_mul(T& a, T& b, T& c, T& d, T e, T f, T g, T h) {
  // [a b; c d] <- [a b; c d] * [e f; g h]
  const T na = a * e + b * g, nb = a * f + b * h, nc = c * e + d * g, nd = c * f + d * h;
  a = na; b = nb; c = nc; d = nd;
}

template <typename T>
__device__ inline void scan_mat2_up_dpp(T& a, T& b, T& c, T& d) {
#define R1S_MSTEP(N)                                \
  {                                                 \
    const T e = dpp<DPP_ROW_SHR + N>(T(1), a);      \
    const T f = dpp<DPP_ROW_SHR + N>(T(0), b);      \
    const T g_ = dpp<DPP_ROW_SHR + N>(T(0), c);     \
    const T h = dpp<DPP_ROW_SHR + N>(T(1), d);      \
    mat2_mul(a, b, c, d, e, f, g_, h);              \
  }
  R1S_MSTEP(1) R1S_MSTEP(2) R1S_MSTEP(4) R1S_MSTEP(8)
#undef R1S_MSTEP
  const T a0 = readlane(a, 15), b0 = readlane(b, 15), c0 = readlane(c, 15), d0 = readlane(d, 15);
  T a1 = readlane(a, 31), b1 = readlane(b, 31), c1 = readlane(c, 31), d1 = readlane(d, 31);
  T a2 = readlane(a, 47), b2 = readlane(b, 47), c2 = readlane(c, 47), d2 = readlane(d, 47);
  // products entering rows 1, 2, 3
  mat2_mul(a1, b1, c1, d1, a0, b0, c0, d0);  // R1 R0
  mat2_mul(a2, b2, c2, d2, a1, b1, c1, d1);  // R2 R1 R0
  const int row = lane_id() >> 4;
  const T pa = row == 0 ? T(1) : row == 1 ? a0 : row == 2 ? a1 : a2;
  const T pb = row == 0 ? T(0) : row == 1 ? b0 : row == 2 ? b1 : b2;
  const T pc = row == 0 ? T(0) : row == 1 ? c0 : row == 2 ? c1 : c2;
  const T pd = row == 0 ? T(1) : row == 1 ? d0 : row == 2 ? d1 : d2;
  mat2_mul(a, b, c, d, pa, pb, pc, pd);
}

// The two bidiagonal sweeps of the SMW local solve over NCH chunks of 64
// unknowns held by one wave, then the 3 x 3 flow corner.
//   forward  y_k = A_k y_{k-1} + (TRANS ? DI_k R_k : R_k)
//   backward x_k = B_k x_{k+1} + (TRANS ? y_k : DI_k y_k)
//   flow lanes x_{L+i} = A rf0 + DI rf1 + B rf2 (the lane's corner-inverse row)
template <typename T, int NCH, bool TRANS>
__device__ inline void smw_sweeps(int L, int m, const T (&A)[NCH], const T (&DI)[NCH],
                                  const T (&B)[NCH], const T (&R)[NCH], T rf0, T rf1, T rf2,
                                  T (&X0)[NCH]) {
  const int lane = lane_id();
  T Y[NCH];
  T carry = T(0);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    const bool lev = k < L;
    T a = lev ? A[ch] : T(0);
    T bb = lev ? (TRANS ? DI[ch] * R[ch] : R[ch]) : T(0);
    if (ch * WAVE < L) {
      scan_affine_up_dpp(a, bb);
      Y[ch] = bb + a * carry;
      carry = readlane(Y[ch], WAVE - 1);
    } else {
      Y[ch] = T(0);
    }
  }
  carry = T(0);
#pragma unroll
  for (int ch = NCH - 1; ch >= 0; --ch) {
    const int k = ch * WAVE + lane;
    const bool lev = k < L;
    T a = lev ? B[ch] : T(0);
    T bb = lev ? (TRANS ? Y[ch] : DI[ch] * Y[ch]) : T(0);
    T x0;
    if (ch * WAVE < L) {
      scan_affine_down_dpp(a, bb);
      x0 = bb + a * carry;
      carry = readlane(x0, 0);
    } else {
      x0 = T(0);
    }
    const T xf = A[ch] * rf0 + DI[ch] * rf1 + B[ch] * rf2;
    X0[ch] = lev ? x0 : (k < m ? xf : T(0));
  }
}

// The sweeps of smw_sweeps for NR right-hand sides of one single-chunk cell
// (m <= 64).  The coefficient half of each affine scan (the products of A or
// B within a row of 16 lanes, and the row prefixes) is the same for every
// right-hand side, so it is formed once; each right-hand side then takes
// only its own half.  The operations, and their order, are those of
// smw_sweeps (the results agree with it to rounding).
template <typename T, int NR, bool TRANS>
__device__ inline void smw_sweeps_nr(int L, int m, T A, T DI, T B, const T (&R)[NR][1],
                                     const T (&RF)[NR][3], T (&X0)[NR][1]) {
  const int lane = lane_id();
  const bool lev = lane < L;
  const int row = lane >> 4;
  T Y[NR];
  {  // forward: y_k = A_k y_{k-1} + (TRANS ? DI_k R_k : R_k)
    T a = lev ? A : T(0);
    T as[4];
#define R1S_STAGE(S, N)                         \
    as[S] = a;                                  \
    a = a * dpp<DPP_ROW_SHR + N>(T(1), a);
    R1S_STAGE(0, 1) R1S_STAGE(1, 2) R1S_STAGE(2, 4) R1S_STAGE(3, 8)
#undef R1S_STAGE
    const T a1 = readlane(a, 31), a2 = readlane(a, 47);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T b = lev ? (TRANS ? DI * R[r][0] : R[r][0]) : T(0);
      b = as[0] * dpp<DPP_ROW_SHR + 1>(T(0), b) + b;
      b = as[1] * dpp<DPP_ROW_SHR + 2>(T(0), b) + b;
      b = as[2] * dpp<DPP_ROW_SHR + 4>(T(0), b) + b;
      b = as[3] * dpp<DPP_ROW_SHR + 8>(T(0), b) + b;
      const T b0 = readlane(b, 15), b1 = readlane(b, 31), b2 = readlane(b, 47);
      const T pb1 = b0;
      const T pb2 = a1 * pb1 + b1;
      const T pb3 = a2 * pb2 + b2;
      const T pb = row == 0 ? T(0) : row == 1 ? pb1 : row == 2 ? pb2 : pb3;
      Y[r] = a * pb + b;
    }
  }
  {  // backward: x_k = B_k x_{k+1} + (TRANS ? y_k : DI_k y_k); flow lanes
    T a = lev ? B : T(0);
    T as[4];
#define R1S_STAGE(S, N)                         \
    as[S] = a;                                  \
    a = a * dpp<DPP_ROW_SHL + N>(T(1), a);
    R1S_STAGE(0, 1) R1S_STAGE(1, 2) R1S_STAGE(2, 4) R1S_STAGE(3, 8)
#undef R1S_STAGE
    const T a2 = readlane(a, 32), a1 = readlane(a, 16);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T b = lev ? (TRANS ? Y[r] : DI * Y[r]) : T(0);
      b = as[0] * dpp<DPP_ROW_SHL + 1>(T(0), b) + b;
      b = as[1] * dpp<DPP_ROW_SHL + 2>(T(0), b) + b;
      b = as[2] * dpp<DPP_ROW_SHL + 4>(T(0), b) + b;
      b = as[3] * dpp<DPP_ROW_SHL + 8>(T(0), b) + b;
      const T b3 = readlane(b, 48), b2 = readlane(b, 32), b1 = readlane(b, 16);
      const T sb2 = b3;
      const T sb1 = a2 * sb2 + b2;
      const T sb0 = a1 * sb1 + b1;
      const T sb = row == 3 ? T(0) : row == 2 ? sb2 : row == 1 ? sb1 : sb0;
      const T x0 = a * sb + b;
      const T xf = A * RF[r][0] + DI * RF[r][1] + B * RF[r][2];
      X0[r][0] = lev ? x0 : (lane < m ? xf : T(0));
    }
  }
}

// Element k of a cell vector held by one wave as NCH chunks of 64 lanes
// (chunk k / 64, lane k % 64), returned wave-uniform; k is wave-uniform.
template <typename T, int NCH>
__device__ inline T lane_value(const T (&v)[NCH], int k) {
  const int kc = k / WAVE, kl = k % WAVE;
  T out = T(0);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
    if (ch == kc) out = readlane(v[ch], kl);
  return out;
}

// Level/flow coupling on a tridiagonal level band, A0 = [T Ec; Er F]: the
// block solve by the Schur complement of the flow unknowns, S3 = F - Er
// T^{-1} Ec.  On entry X0 holds the sweeps' output: T^{-1} r on the level
// lanes, S3^{-1} r_F on the flow lanes (the lane's S3^{-1} row sits in the
// flow lanes of A, DI, B).  With t = Er (T^{-1} r_L): x_F = S3^{-1} (r_F -
// t) and x_L = T^{-1} r_L - X x_F, X = T^{-1} Ec (rows X[i], zero past the
// levels; E[i] the coupling rows Er, zero past the levels).  The transposed
// solve uses the same steps on A0^T = [T^T Er^T; Ec^T F^T].
template <typename T, int NCH>
__device__ inline void arrow_schur(int L, int m, const T (&A)[NCH], const T (&DI)[NCH],
                                   const T (&B)[NCH], const T (&X)[3][NCH], const T (&E)[3][NCH],
                                   T (&X0)[NCH]) {
  const int lane = lane_id();
  T t[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T s = T(0);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) s += ch * WAVE + lane < L ? E[i][ch] * X0[ch] : T(0);
    t[i] = wave_sum_u(s);
  }
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int k = ch * WAVE + lane;
    if (k >= L && k < m) X0[ch] -= A[ch] * t[0] + DI[ch] * t[1] + B[ch] * t[2];
  }
  T z[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) z[i] = lane_value<T, NCH>(X0, L + i);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
    if (ch * WAVE + lane < L) X0[ch] -= X[0][ch] * z[0] + X[1][ch] * z[1] + X[2][ch] * z[2];
}

// Per-cell inverse capacitance C^{-1} of the Woodbury correction.  With one
// pair it is a scalar per cell; with rd pairs lane t of the wave holds entries t and
// 64 + t of the cell's row-major C^{-1} (rd^2 <= 81 values), read back with
// v_readlane (transposed apply: (C^{-1})^T, the same values read transposed).
template <typename TV, int RDM>
struct CapInv {
  static constexpr int NV = (RDM * RDM + WAVE - 1) / WAVE;
  TV v[NV];
  __device__ inline void load(const TV* invC, int c, int rd, int lane) {
    if (RDM == 1) {
      v[0] = invC[c];
    } else {
      const int cnt = rd * rd;
      const TV* p = invC + (long long)c * cnt;
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const int t = h * WAVE + lane;
        v[h] = p[t < cnt ? t : cnt - 1];
      }
    }
  }
  // z_i = sum_l Cinv(i, l) s_l   (TRANS: Cinv(l, i))
  template <bool TRANS>
  __device__ inline void apply(const TV (&s)[RDM], TV (&z)[RDM], int rd) const {
    if (RDM == 1) {
      z[0] = s[0] * v[0];
      return;
    }
#pragma unroll
    for (int i = 0; i < RDM; ++i) {
      TV acc = TV(0);
#pragma unroll
      for (int l = 0; l < RDM; ++l) {
        if (i < rd && l < rd) {
          const int t = TRANS ? l * rd + i : i * rd + l;
          const TV e = t < WAVE ? readlane(v[0], t) : readlane(v[NV - 1], t - (NV - 1) * WAVE);
          acc += e * s[l];
        }
      }
      z[i] = acc;
    }
  }
};

// ----------------------------------------- wide diagonal-block pattern ----
// Terms of S_cc beyond the tridiagonal band and the 3x3 corner: the level
// diagonals j = 2..band and the level/flow coupling.  Forward, lane k adds
// row k; transposed, column k (the band entries of rows k -+ j).
//
// Coupling rows dotted with the cell's levels (a wave sum per flow unknown):
// forward the flow rows S[L+i][.] (fa + 3 + i), transposed the flow columns
// S[.][L+i] (fa + i).  Per-lane coupling rows times x_{L+i}: forward
// S[k][L+i] (fa + i), transposed S[L+i][k] (fa + 3 + i).
// Slot 3 (the atom) the same way, with x_a and lane a in place of x_{L+i}
// and lane L + i.
template <bool TRANS>
__device__ inline int arrow_sum_row(const Mesh& g, int i) {
  return TRANS ? arrow_col_row(g, i) : arrow_row_row(g, i);
}
template <bool TRANS>
__device__ inline int arrow_lane_row(const Mesh& g, int i) {
  return TRANS ? arrow_row_row(g, i) : arrow_col_row(g, i);
}

// The coupling slots of either kind of wide diagonal block: the structured
// layouts' (WIDE = 1: flow unknowns, atom) or a general pattern's dense
// indices (WIDE = 2: column row fa + i, row row fa + ns + i, index px[i]).
template <int WIDE, bool TRANS>
__device__ inline int slot_sum_row(const Mesh& g, int i) {
  if constexpr (WIDE == 2) return TRANS ? g.fa + i : g.fa + g.ns + i;
  else return arrow_sum_row<TRANS>(g, i);
}
template <int WIDE, bool TRANS>
__device__ inline int slot_lane_row(const Mesh& g, int i) {
  if constexpr (WIDE == 2) return TRANS ? g.fa + g.ns + i : g.fa + i;
  else return arrow_lane_row<TRANS>(g, i);
}
template <int WIDE>
__device__ inline int slot_x(const Mesh& g, int i) {
  if constexpr (WIDE == 2) return g.px[i];
  else return arrow_unknown(g.L, i);
}

// The ELL entries of a general pattern at lane kk: forward, row kk's entries
// (record rows fb + s, columns from the shared table); transposed, column
// kk's entries (values gathered from the record by offset, their rows from
// the table).  Absent entries get a zero value and the lane's own index.
template <typename TV, bool TRANS>
struct PatLane {
  TV a[PAT_ELL_MAX];
  int col[PAT_ELL_MAX];

  __device__ inline void load(const Mesh& g, const TV* rc, int kk) {
    const long long mp = g.mp;
    const int n = TRANS ? g.net : g.ne;
    // the lane's packed columns (forward) or slot/row halfwords (transposed)
    unsigned w[PAT_ELL_MAX / 2];
    if (TRANS) {
      const uint4* t = reinterpret_cast<const uint4*>(g.ptpos + kk * (PAT_ELL_MAX / 2));
      const uint4 t0 = t[0], t1 = t[1];
      w[0] = t0.x; w[1] = t0.y; w[2] = t0.z; w[3] = t0.w;
      w[4] = t1.x; w[5] = t1.y; w[6] = t1.z; w[7] = t1.w;
    } else {
      const uint4 c = *reinterpret_cast<const uint4*>(g.pcol + kk * (PAT_ELL_MAX / 4));
      w[0] = c.x; w[1] = c.y; w[2] = c.z; w[3] = c.w;
    }
#pragma unroll
    for (int s = 0; s < PAT_ELL_MAX; ++s) {
      a[s] = TV(0);
      col[s] = kk;
      if (s < n) {
        if (TRANS) {
          const unsigned h = (w[s >> 1] >> (16 * (s & 1))) & 0xffffu;
          const bool on = h != 0xffffu;
          col[s] = on ? (int)(h & 0xffu) : kk;
          a[s] = on ? rc[(g.fb + (int)(h >> 8)) * mp + (h & 0xffu)] : TV(0);
        } else {
          a[s] = rc[(g.fb + s) * mp + kk];
          col[s] = (int)((w[s >> 2] >> (8 * (s & 3))) & 0xffu);
        }
      }
    }
  }
  // (guards instead of an early exit, so that the loops unroll and the
  // slots stay in registers)
  __device__ inline TV apply(const Mesh& g, const double* xc) const {
    const int n = TRANS ? g.net : g.ne;
    TV s = TV(0);
#pragma unroll
    for (int t = 0; t < PAT_ELL_MAX; ++t)
      if (t < n) s += a[t] * (TV)xc[col[t]];
    return s;
  }
  __device__ inline TV apply_lanes(const Mesh& g, TV xk) const {
    const int n = TRANS ? g.net : g.ne;
    TV s = TV(0);
#pragma unroll
    for (int t = 0; t < PAT_ELL_MAX; ++t)
      if (t < n) s += a[t] * __shfl(xk, col[t], WAVE);
    return s;
  }
};

// Band coefficients of lane kk (clamped lane index) and the x indices they
// multiply; invalid positions get a zero coefficient and a valid index.
template <typename TV, bool TRANS>
struct BandLane {
  TV alo[BAND_MAX - 1], ahi[BAND_MAX - 1];
  int ilo[BAND_MAX - 1], ihi[BAND_MAX - 1];

  __device__ inline void load(const Mesh& g, const TV* rc, int kk) {
    const long long mp = g.mp;
    const int L = g.L, nbd = g.band - 1;
#pragma unroll
    for (int j = 2; j <= BAND_MAX; ++j) {
      const int t = j - 2;
      const bool on = j <= g.band;
      const bool vlo = on && kk < L && kk >= j;  // x_{k-j}: S[k][k-j] or S[k-j][k]
      const bool vhi = on && kk + j < L;         // x_{k+j}: S[k][k+j] or S[k+j][k]
      ilo[t] = vlo ? kk - j : kk;
      ihi[t] = vhi ? kk + j : kk;
      TV a = TV(0), b = TV(0);
      if (on) {
        // forward: lower row j at k, upper row j at k; transposed: upper row
        // j at k - j (entry S[k-j][k]), lower row j at k + j (S[k+j][k])
        a = TRANS ? rc[(g.fb + nbd + t) * mp + ilo[t]] : rc[(g.fb + t) * mp + kk];
        b = TRANS ? rc[(g.fb + t) * mp + ihi[t]] : rc[(g.fb + nbd + t) * mp + kk];
      }
      alo[t] = vlo ? a : TV(0);
      ahi[t] = vhi ? b : TV(0);
    }
  }
  __device__ inline TV apply(const Mesh& g, const double* xc) const {
    TV s = TV(0);
#pragma unroll
    for (int t = 0; t < BAND_MAX - 1; ++t) {
      if (t + 2 > g.band) break;
      s += alo[t] * (TV)xc[ilo[t]] + ahi[t] * (TV)xc[ihi[t]];
    }
    return s;
  }
  // The same with the cell's x block held one element per lane (m <= 64):
  // the partners come from the lanes that hold them.
  __device__ inline TV apply_lanes(const Mesh& g, TV xk) const {
    TV s = TV(0);
#pragma unroll
    for (int t = 0; t < BAND_MAX - 1; ++t) {
      if (t + 2 > g.band) break;
      s += alo[t] * __shfl(xk, ilo[t], WAVE) + ahi[t] * __shfl(xk, ihi[t], WAVE);
    }
    return s;
  }
};

// The lane terms of the wide diagonal block of either kind.
template <typename TV, bool TRANS, int WIDE>
struct DiagLaneSel {
  using type = BandLane<TV, TRANS>;
};
template <typename TV, bool TRANS>
struct DiagLaneSel<TV, TRANS, 2> {
  using type = PatLane<TV, TRANS>;
};
template <typename TV, bool TRANS, int WIDE>
using DiagLane = typename DiagLaneSel<TV, TRANS, WIDE>::type;

}  // namespace r1s
