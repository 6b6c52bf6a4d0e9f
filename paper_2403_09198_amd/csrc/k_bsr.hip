// Dense-block BSR baseline: the standard representation of section 3
// (Jacobian Complexity, N_A = sum m^2 (N_e + 1) stored values) in the BSR
// format of section 5.1, and the classical block-Jacobi of section 6 (LU of
// every dense diagonal block).
//
// Blocks are stored column-major (element (i, j) of block b at b*m*m + j*m + i)
// so that the lanes of a wavefront, one per block row i, read contiguous
// memory for every column j.
#include <math.h>

#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

// D_{c,d} = S_{c,d} + sum_p u_p v_p^T, one workgroup per block.
__global__ __launch_bounds__(256) void k_bsr_assemble(Mesh g, const double* __restrict__ rec,
                                                      const int* __restrict__ blk_row,
                                                      const int* __restrict__ blk_dir,
                                                      double* __restrict__ data) {
  const long long b = blockIdx.x;
  const int c = blk_row[b], d = blk_dir[b];
  const int m = g.m, mp = g.mp, L = g.L;
  const double* rc = rec + (long long)c * g.F * mp;
  const double* u = rc + (long long)(g.fu + pair_start(g, d)) * mp;         // pair p at + p mp
  const double* v = rc + (long long)(g.fu + g.P + pair_start(g, d)) * mp;
  const int cnt = pair_count(g, d);
  double* out = data + b * m * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int j = e / m, i = e - j * m;
    double s = 0.0;
    if (d == D_C && g.pat) {  // general pattern: the entry at (i, j), if any
      const int en = g.pdense[i * m + j];
      s = en >= 0 ? rc[g.peoff[en]] : 0.0;
    } else if (d == D_C) {
      if (i == j) {
        s = rc[F_DIAG * mp + i];
      } else if (i < L && j < L) {
        if (j == i - 1) s = rc[F_LO * mp + i];
        if (j == i + 1) s = rc[F_HI * mp + i];
      } else if (i >= L && j >= L) {
        const int a = i - L, bb = j - L;
        if (bb == (a + 2) % 3) s = rc[F_LO * mp + i];
        if (bb == (a + 1) % 3) s = rc[F_HI * mp + i];
      }
      // wide pattern: level diagonals j = 2..band and the level/flow coupling
      if (i < L && j < L && i != j) {
        const int dd = i - j, nbd = g.band - 1;
        if (dd >= 2 && dd <= g.band) s = rc[(g.fb + dd - 2) * mp + i];
        if (-dd >= 2 && -dd <= g.band) s = rc[(g.fb + nbd - dd - 2) * mp + i];
      } else if (g.arrow && i < L && j >= L) {
        s = rc[(g.fa + j - L) * mp + i];
      } else if (g.arrow && i >= L && j < L) {
        s = rc[(g.fa + 3 + i - L) * mp + j];
      }
      // the atom's column and row, added to what the band holds there
      if (g.arrow == 2) {
        const int a = L - 1;
        if (j == a && i < a) s += rc[(long long)arrow_col_row(g, 3) * mp + i];
        if (i == a && j < a) s += rc[(long long)arrow_row_row(g, 3) * mp + j];
      }
    } else if (i == j) {
      s = rc[nbr_row(g, d) * mp + i];
    }
    for (int p = 0; p < cnt; ++p) s += u[p * mp + i] * v[p * mp + j];
    out[e] = s;
  }
}

hipError_t launch_bsr_assemble(const Mesh& g, const double* rec, const int* blk_row,
                               const int* blk_dir, long long nblocks, double* data,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_bsr_assemble, dim3((unsigned)nblocks), dim3(256), 0, s, g, rec, blk_row,
                     blk_dir, data);
  return hipGetLastError();
}

// y_c = sum_b D_b x_{col(b)}.  One wavefront per (cell, 64-row chunk); the
// column blocks of x are read as wave-uniform values.
__global__ __launch_bounds__(256) void k_bsr_matvec(Mesh g, const int* __restrict__ indptr,
                                                    const int* __restrict__ indices,
                                                    const double* __restrict__ data,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y, int nrhs) {
  const int nch = (g.m + WAVE - 1) / WAVE;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int unit = __builtin_amdgcn_readfirstlane(tile * 4 + (int)(threadIdx.x >> 6));
  if (unit >= g.N * nch) return;
  const int c = unit / nch, ch = unit - c * nch;
  const int m = g.m;
  const int i = ch * WAVE + lane_id();
  const bool act = i < m;
  const int b0 = indptr[c], b1 = indptr[c + 1];
  for (int r = 0; r < nrhs; ++r) {
    double acc = 0.0;
    for (int b = b0; b < b1; ++b) {
      const double* D = data + (long long)b * m * m + i;
      const double* xc = x + (long long)r * g.n + (long long)indices[b] * m;
      int j = 0;
      for (; j + 4 <= m; j += 4) {
        const double d0 = act ? D[(long long)(j + 0) * m] : 0.0;
        const double d1 = act ? D[(long long)(j + 1) * m] : 0.0;
        const double d2 = act ? D[(long long)(j + 2) * m] : 0.0;
        const double d3 = act ? D[(long long)(j + 3) * m] : 0.0;
        acc += d0 * xc[j] + d1 * xc[j + 1] + d2 * xc[j + 2] + d3 * xc[j + 3];
      }
      for (; j < m; ++j) acc += (act ? D[(long long)j * m] : 0.0) * xc[j];
    }
    if (act) y[(long long)r * g.n + (long long)c * m + i] = acc;
  }
}

hipError_t launch_bsr_matvec(const Mesh& g, const int* indptr, const int* indices,
                             const double* data, const double* x, double* y, int nrhs,
                             hipStream_t s) {
  const int nch = (g.m + WAVE - 1) / WAVE;
  const long long units = (long long)g.N * nch;
  hipLaunchKernelGGL(k_bsr_matvec, dim3((unsigned)((units + 3) / 4)), dim3(256), 0, s, g, indptr,
                     indices, data, x, y, nrhs);
  return hipGetLastError();
}

// LU with partial pivoting of the diagonal block of every cell, one
// workgroup per cell, right-looking elimination on a column-major copy in
// LDS (m*m*8 <= 64 KiB, i.e. m <= 90).  Larger blocks go to the batched
// library LU (see the BSR preconditioner setup).
template <bool IN_LDS>
__global__ __launch_bounds__(256) void k_bsr_lu(Mesh g, const int* __restrict__ diag_block,
                                                const double* __restrict__ data,
                                                double* __restrict__ lu, int* __restrict__ piv,
                                                int* status) {
  extern __shared__ double smem[];
  __shared__ double red_v[4];
  __shared__ int red_i[4];
  __shared__ int s_p;
  const int c = blockIdx.x;
  const int m = g.m;
  const long long mm = (long long)m * m;
  const double* src = data + (long long)diag_block[c] * mm;
  double* out = lu + (long long)c * mm;
  double* A = IN_LDS ? smem : out;
  for (int e = threadIdx.x; e < mm; e += blockDim.x) A[e] = src[e];
  __syncthreads();
  bool bad = false;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  for (int k = 0; k < m; ++k) {
    // pivot: argmax |A[i][k]|, i >= k (lowest index on ties)
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < m; i += blockDim.x) {
      const double a = fabs(A[(long long)k * m + i]);
      if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, WAVE);
      const int oi = __shfl_xor(bi, off, WAVE);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { red_v[wave] = best; red_i[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = red_v[0];
      int bidx = red_i[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bidx)) { bv = red_v[w]; bidx = red_i[w]; }
      s_p = bidx;
      piv[(long long)c * m + k] = bidx;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double t = A[(long long)j * m + k];
        A[(long long)j * m + k] = A[(long long)j * m + p];
        A[(long long)j * m + p] = t;
      }
    __syncthreads();
    const double pv = A[(long long)k * m + k];
    if (pv == 0.0) bad = true;
    const double pinv = 1.0 / pv;
    for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) A[(long long)k * m + i] *= pinv;
    __syncthreads();
    const int nt = m - k - 1;
    for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
      const int jj = e / nt, ii = e - jj * nt;
      const int i = k + 1 + ii, j = k + 1 + jj;
      A[(long long)j * m + i] -= A[(long long)k * m + i] * A[(long long)j * m + k];
    }
    __syncthreads();
  }
  if (IN_LDS)
    for (int e = threadIdx.x; e < mm; e += blockDim.x) out[e] = A[e];
  if (bad && threadIdx.x == 0) atomicMin(status, c);
}

bool bsr_lu_fits_lds(const Mesh& g) { return (size_t)g.m * g.m * sizeof(double) <= 65536; }

hipError_t launch_bsr_lu_setup(const Mesh& g, const int* diag_block, const double* data,
                               double* lu, int* piv, int* status, hipStream_t s) {
  if (!bsr_lu_fits_lds(g)) return hipErrorInvalidValue;
  const size_t lds = (size_t)g.m * g.m * sizeof(double);
  hipLaunchKernelGGL(k_bsr_lu<true>, dim3(g.N), dim3(256), lds, s, g, diag_block, data, lu, piv,
                     status);
  return hipGetLastError();
}

// Copies the diagonal block of every cell into lu[c] (the in-place input of
// the batched library LU used for blocks that do not fit in LDS).
__global__ __launch_bounds__(256) void k_bsr_gather_diag(Mesh g, const int* __restrict__ diag_block,
                                                         const double* __restrict__ data,
                                                         double* __restrict__ lu) {
  const long long mm = (long long)g.m * g.m;
  const double* src = data + (long long)diag_block[blockIdx.x] * mm;
  double* dst = lu + (long long)blockIdx.x * mm;
  for (long long e = threadIdx.x; e < mm; e += blockDim.x) dst[e] = src[e];
}

// 1-based LAPACK pivots -> 0-based; info > 0 (exact zero pivot) -> status.
__global__ __launch_bounds__(256) void k_bsr_piv_convert(Mesh g, int* __restrict__ piv,
                                                         const int* __restrict__ info,
                                                         int* status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (long long)g.N * g.m) piv[i] -= 1;
  if (i < g.N && info[i] != 0) atomicMin(status, (int)i);
}

hipError_t launch_bsr_gather_diag(const Mesh& g, const int* diag_block, const double* data,
                                  double* lu, hipStream_t s) {
  hipLaunchKernelGGL(k_bsr_gather_diag, dim3(g.N), dim3(256), 0, s, g, diag_block, data, lu);
  return hipGetLastError();
}

hipError_t launch_bsr_piv_convert(const Mesh& g, int* piv, const int* info, int* status,
                                  hipStream_t s) {
  const long long n = (long long)g.N * g.m;
  hipLaunchKernelGGL(k_bsr_piv_convert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, piv,
                     info, status);
  return hipGetLastError();
}

// z_c = D_cc^{-1} r_c from the packed LU: row swaps, unit-lower forward
// substitution, upper back substitution.  One wavefront per cell; the m
// unknowns sit in NCH registers per lane.  Columns of the factors are loaded
// JB at a time ahead of the dependent substitution steps, and each newly
// final unknown is broadcast with v_readlane.
template <int NCH>
__device__ inline double bcast(const double (&y)[NCH], int j) {
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < NCH; ++s)
    if (s == (j >> 6)) v = readlane(y[s], j & 63);
  return v;
}

template <int NCH>
__global__ __launch_bounds__(256) void k_bsr_lu_apply(Mesh g, const double* __restrict__ lu,
                                                      const int* __restrict__ piv,
                                                      const double* __restrict__ rin,
                                                      double* __restrict__ zout, int nrhs) {
  constexpr int JB = 16;
  const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  if (c >= g.N) return;
  const int lane = lane_id();
  const int m = g.m;
  const double* LU = lu + (long long)c * m * m;
  const int* P = piv + (long long)c * m;
  int pv[NCH];
#pragma unroll
  for (int s = 0; s < NCH; ++s) {
    const int i = s * WAVE + lane;
    pv[s] = P[i < m ? i : m - 1];
  }
  for (int r = 0; r < nrhs; ++r) {
    const double* rv = rin + (long long)r * g.n + (long long)c * m;
    double y[NCH];
#pragma unroll
    for (int s = 0; s < NCH; ++s) {
      const int i = s * WAVE + lane;
      y[s] = rv[i < m ? i : m - 1];
    }
    // row swaps in order
    for (int k = 0; k < m; ++k) {
      int p = 0;
#pragma unroll
      for (int s = 0; s < NCH; ++s)
        if (s == (k >> 6)) p = __builtin_amdgcn_readlane(pv[s], k & 63);
      if (p == k) continue;
      const double vk = bcast(y, k), vp = bcast(y, p);
#pragma unroll
      for (int s = 0; s < NCH; ++s) {
        const int i = s * WAVE + lane;
        if (i == k) y[s] = vp;
        if (i == p) y[s] = vk;
      }
    }
    // forward: unit lower triangle
    for (int j0 = 0; j0 < m; j0 += JB) {
      double col[JB][NCH];
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const int j = j0 + t < m ? j0 + t : m - 1;
#pragma unroll
        for (int s = 0; s < NCH; ++s) {
          const int i = s * WAVE + lane;
          col[t][s] = LU[(long long)j * m + (i < m ? i : m - 1)];
        }
      }
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const int j = j0 + t;
        if (j >= m) break;
        const double yj = bcast(y, j);
#pragma unroll
        for (int s = 0; s < NCH; ++s) {
          const int i = s * WAVE + lane;
          if (i > j && i < m) y[s] -= col[t][s] * yj;
        }
      }
    }
    // backward: upper triangle
    for (int j1 = m - 1; j1 >= 0; j1 -= JB) {
      double col[JB][NCH];
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const int j = j1 - t >= 0 ? j1 - t : 0;
#pragma unroll
        for (int s = 0; s < NCH; ++s) {
          const int i = s * WAVE + lane;
          col[t][s] = LU[(long long)j * m + (i < m ? i : m - 1)];
        }
      }
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const int j = j1 - t;
        if (j < 0) break;
        const double dj = LU[(long long)j * m + j];
        const double xj = bcast(y, j) / dj;
#pragma unroll
        for (int s = 0; s < NCH; ++s) {
          const int i = s * WAVE + lane;
          if (i == j) y[s] = xj;
          if (i < j) y[s] -= col[t][s] * xj;
        }
      }
    }
    double* zv = zout + (long long)r * g.n + (long long)c * m;
#pragma unroll
    for (int s = 0; s < NCH; ++s) {
      const int i = s * WAVE + lane;
      if (i < m) zv[i] = y[s];
    }
  }
}

hipError_t launch_bsr_lu_apply(const Mesh& g, const double* lu, const int* piv, const double* r,
                               double* z, int nrhs, hipStream_t s) {
  const int grid = (g.N + 3) / 4;
  switch ((g.m + WAVE - 1) / WAVE) {
    case 1: hipLaunchKernelGGL(k_bsr_lu_apply<1>, dim3(grid), dim3(256), 0, s, g, lu, piv, r, z, nrhs); break;
    case 2: hipLaunchKernelGGL(k_bsr_lu_apply<2>, dim3(grid), dim3(256), 0, s, g, lu, piv, r, z, nrhs); break;
    case 3: hipLaunchKernelGGL(k_bsr_lu_apply<3>, dim3(grid), dim3(256), 0, s, g, lu, piv, r, z, nrhs); break;
    case 4: hipLaunchKernelGGL(k_bsr_lu_apply<4>, dim3(grid), dim3(256), 0, s, g, lu, piv, r, z, nrhs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace r1s
