// Device-side helpers shared by the r1s kernels (gfx950, wave64).
//
// Internal layout of the packed Jacobian ("record" layout): one contiguous
// record per mesh cell, [N][F][mp] values, F = 17 field rows of mp = m
// rounded up to a multiple of 8 (64-byte rows).  Lane k of the wave that owns
// cell c reads element k of every row, so every load is one contiguous run.
//
//   row 0      diag    S_cc[k][k]
//   row 1      lo      level k: S_cc[k][k-1]; flow row i: S_cc[L+i][L+(i+2)%3]
//   row 2      hi      level k: S_cc[k][k+1]; flow row i: S_cc[L+i][L+(i+1)%3]
//   rows 3..6  nbr     diagonal of S_{c,d}, d = S, W, E, N
//   rows 7..11 u       u_{c,d}, d = S, W, C, E, N
//   rows 12..16 v      v_{c,d}, d = S, W, C, E, N
//
// Padding elements and the rows of blocks that do not exist (mesh boundary)
// are zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace r1s {

constexpr int WAVE = 64;
constexpr int NXCD = 8;      // MI355X: 8 XCDs x 32 CUs
constexpr int F_REC = 17;    // field rows per cell record
constexpr int F_DIAG = 0, F_LO = 1, F_HI = 2, F_NBR = 3, F_U = 7, F_V = 12;
constexpr int D_S = 0, D_W = 1, D_C = 2, D_E = 3, D_N = 4;
constexpr int MAX_CHUNKS = 4;  // m <= 256

// SMW factor records, [N][5][mp] per direction of application.
//   forward:   a = -l_k,  dinv = 1/d_k,  b = -s_k/d_k,  w = S_cc^{-1} u_cC, v_cC
//   transpose: a = -s_{k-1}/d_k, dinv, b = -l_{k+1},  wt = S_cc^{-T} v_cC, u_cC
// Flow lanes L+i hold row i of the 3x3 corner inverse (transpose: of its
// transpose) in the a / dinv / b rows.
constexpr int F_SMW = 5;
constexpr int P_A = 0, P_DINV = 1, P_B = 2, P_W = 3, P_V = 4;

__host__ __device__ inline int pad_m(int m) { return (m + 7) & ~7; }
__host__ __device__ inline int nbr_slot(int d) { return d < 2 ? d : d - 1; }
__host__ __device__ inline int opposite(int d) { return 4 - d; }

struct Mesh {
  int nx, ny, L, m, mp;
  int N;           // nx*ny
  long long n;     // N*m, stride between right-hand sides
};

// Workgroup id -> logical tile, so that each XCD (which receives every
// NXCD-th workgroup) works on one contiguous range of tiles and keeps the
// neighbouring x blocks in its own L2.
__device__ inline int xcd_tile(int bid, int grid) {
  const int xcd = bid % NXCD, local = bid / NXCD;
  const int per = grid / NXCD, rem = grid % NXCD;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }

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

}  // namespace r1s
