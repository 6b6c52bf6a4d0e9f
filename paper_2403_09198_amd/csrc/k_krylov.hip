// Float64 vector kernels of restarted GMRES: Gram-Schmidt dot products with
// a deterministic two-stage reduction (fixed block partials, then a fixed-order
// sum per row), basis updates, normalisation and the final combination.
// All right-hand sides advance together: blockIdx.y (or a loop) selects the
// right-hand side.
#include <math.h>

#include "r1s_device.hpp"
#include "r1s_kernels.hpp"

namespace r1s {

constexpr int KB = 256;  // threads per block of the vector kernels

int dot_blocks(long long n) {
  long long b = (n + 8LL * KB - 1) / (8LL * KB);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < KB / WAVE; ++w) t += sh[w];
  return t;
}

// part[((r*(nv+1)) + i)*nblk + blk] = sum over this block's elements of
// V_i . w   (i < nv), and w . w at i = nv when with_norm.
__global__ __launch_bounds__(KB) void k_multidot(Basis B, int nv, const double* __restrict__ w,
                                                 long long wstride, long long n,
                                                 double* __restrict__ part, int nblk,
                                                 int with_norm) {
  __shared__ double sh[KB / WAVE];
  const int r = blockIdx.y;
  const double* wr = w + (long long)r * wstride;
  const double* Vr = B.V + (long long)r * B.rstride;
  const long long stride = (long long)nblk * KB;
  const long long e0 = (long long)blockIdx.x * KB + threadIdx.x;
  double* pr = part + (long long)r * (nv + 1) * nblk;
  int i = 0;
  for (; i + 4 <= nv; i += 4) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    const double* v0 = Vr + (long long)i * B.vstride;
    for (long long e = e0; e < n; e += stride) {
      const double we = wr[e];
      a0 += v0[e] * we;
      a1 += v0[e + B.vstride] * we;
      a2 += v0[e + 2 * B.vstride] * we;
      a3 += v0[e + 3 * B.vstride] * we;
    }
    a0 = block_sum(a0, sh); a1 = block_sum(a1, sh);
    a2 = block_sum(a2, sh); a3 = block_sum(a3, sh);
    if (threadIdx.x == 0) {
      pr[(long long)(i + 0) * nblk + blockIdx.x] = a0;
      pr[(long long)(i + 1) * nblk + blockIdx.x] = a1;
      pr[(long long)(i + 2) * nblk + blockIdx.x] = a2;
      pr[(long long)(i + 3) * nblk + blockIdx.x] = a3;
    }
  }
  for (; i < nv; ++i) {
    double a0 = 0;
    const double* v0 = Vr + (long long)i * B.vstride;
    for (long long e = e0; e < n; e += stride) a0 += v0[e] * wr[e];
    a0 = block_sum(a0, sh);
    if (threadIdx.x == 0) pr[(long long)i * nblk + blockIdx.x] = a0;
  }
  if (with_norm) {
    double a0 = 0;
    for (long long e = e0; e < n; e += stride) a0 += wr[e] * wr[e];
    a0 = block_sum(a0, sh);
    if (threadIdx.x == 0) pr[(long long)nv * nblk + blockIdx.x] = a0;
  }
}

hipError_t launch_multidot(Basis B, int nv, const double* w, long long wstride, long long n,
                           int nrhs, double* part, int nblk, bool with_norm, hipStream_t s) {
  hipLaunchKernelGGL(k_multidot, dim3(nblk, nrhs), dim3(KB), 0, s, B, nv, w, wstride, n, part,
                     nblk, (int)with_norm);
  return hipGetLastError();
}

// out[row] = sum_blk part[row*nblk + blk] in a fixed order, one wave per row:
// lane l adds blocks l, l + 64, ... in turn, then the wave sum.  nblk <=
// 1024 (dot_blocks), so each lane holds at most 16 partials, all loaded
// before the first add.
constexpr int REDUCE_PER_LANE = 16;
__global__ __launch_bounds__(KB) void k_reduce(const double* __restrict__ part, int rows, int nblk,
                                               double* __restrict__ out) {
  const int row = blockIdx.x * (KB / WAVE) + (threadIdx.x >> 6);
  if (row >= rows) return;
  const double* pr = part + (long long)row * nblk;
  double v[REDUCE_PER_LANE];
#pragma unroll
  for (int t = 0; t < REDUCE_PER_LANE; ++t) {
    const int b = lane_id() + t * WAVE;
    v[t] = b < nblk ? pr[b] : 0.0;
  }
  double a = 0.0;
#pragma unroll
  for (int t = 0; t < REDUCE_PER_LANE; ++t) a += v[t];
  a = wave_sum(a);
  if (lane_id() == 0) out[row] = a;
}

// k_reduce for a few rows in one workgroup that also hands them to the
// host: out[row] and host[row] (pinned), then flag[0] = seq once host[] is
// visible (see stage_ready).
__global__ __launch_bounds__(KB) void k_reduce_host(const double* __restrict__ part, int rows,
                                                    int nblk, double* __restrict__ out,
                                                    double* host, int* flag, int seq) {
  for (int row = threadIdx.x >> 6; row < rows; row += KB / WAVE) {
    const double* pr = part + (long long)row * nblk;
    double v[REDUCE_PER_LANE];
#pragma unroll
    for (int t = 0; t < REDUCE_PER_LANE; ++t) {
      const int b = lane_id() + t * WAVE;
      v[t] = b < nblk ? pr[b] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < REDUCE_PER_LANE; ++t) a += v[t];
    a = wave_sum(a);
    if (lane_id() == 0) {
      out[row] = a;
      host[row] = a;
    }
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_reduce_host(const double* part, int rows, int nblk, double* out, double* host,
                              int* flag, int seq, hipStream_t s) {
  if (nblk > REDUCE_PER_LANE * WAVE) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_host, dim3(1), dim3(KB), 0, s, part, rows, nblk, out, host, flag,
                     seq);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int rows, int nblk, double* out, hipStream_t s) {
  if (nblk > REDUCE_PER_LANE * WAVE) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3((rows + KB / WAVE - 1) / (KB / WAVE)), dim3(KB), 0, s, part,
                     rows, nblk, out);
  return hipGetLastError();
}

static inline dim3 vec_grid(long long n, int nrhs) {
  long long b = (n + 4LL * KB - 1) / (4LL * KB);
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b, nrhs);
}

// Fused reorthogonalisation pass for small bases (nv <= NVMAX): each thread
// loads V_i[e] once into registers, forms w1[e] = w[e] - sum_i h_i V_i[e],
// stores it, and accumulates V_i[e] w1[e] and w1[e]^2 for the next
// coefficients (partials per block, reduced by k_reduce as for k_multidot).
// The pass runs only where it is needed (Daniel-Gragg-Kaufman-Stewart: the
// first pass left |w - V h|^2 = |w|^2 - |h|^2 <= |w|^2 / 2), or always; the
// decision per right-hand side goes to need[r], and a skipped pass leaves w
// and writes zero partials.
template <int NVMAX>
__global__ __launch_bounds__(KB) void k_update_multidot(Basis B, int nv, const double* __restrict__ h,
                                                        int hstride, double* __restrict__ w,
                                                        long long wstride, long long n,
                                                        double* __restrict__ part, int nblk,
                                                        int always, int* __restrict__ need) {
  __shared__ double sh[KB / WAVE];
  const int r = blockIdx.y;
  const double* Vr = B.V + (long long)r * B.rstride;
  const double* hr = h + (long long)r * hstride;
  double* wr = w + (long long)r * wstride;
  double* pr = part + (long long)r * (nv + 1) * nblk;
  double h2sum = 0.0;
  for (int i = 0; i < nv; ++i) h2sum += hr[i] * hr[i];
  const bool run = always || !(hr[nv] - h2sum > 0.5 * hr[nv]);  // block-uniform
  if (blockIdx.x == 0 && threadIdx.x == 0) need[r] = run ? 1 : 0;
  if (!run) {  // every block of this right-hand side takes this branch
    if (threadIdx.x == 0)
      for (int i = 0; i <= nv; ++i) pr[(long long)i * nblk + blockIdx.x] = 0.0;
    return;
  }
  double hv[NVMAX], acc[NVMAX];
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    hv[i] = i < nv ? hr[i] : 0.0;
    acc[i] = 0.0;
  }
  double accn = 0.0;
  const long long stride = (long long)nblk * KB;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += stride) {
    double v[NVMAX];
    double a = wr[e];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      v[i] = i < nv ? Vr[(long long)i * B.vstride + e] : 0.0;
      a -= hv[i] * v[i];
    }
    wr[e] = a;
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) acc[i] += v[i] * a;
    accn += a * a;
  }
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    if (i >= nv) break;
    const double t = block_sum(acc[i], sh);
    if (threadIdx.x == 0) pr[(long long)i * nblk + blockIdx.x] = t;
  }
  const double t = block_sum(accn, sh);
  if (threadIdx.x == 0) pr[(long long)nv * nblk + blockIdx.x] = t;
}

int update_multidot_max() { return 16; }

hipError_t launch_update_multidot(Basis B, int nv, const double* h, int hstride, double* w,
                                  long long wstride, long long n, int nrhs, double* part, int nblk,
                                  bool always, int* need, hipStream_t s) {
  if (nv <= 8)
    hipLaunchKernelGGL(k_update_multidot<8>, dim3(nblk, nrhs), dim3(KB), 0, s, B, nv, h, hstride,
                       w, wstride, n, part, nblk, (int)always, need);
  else if (nv <= 16)
    hipLaunchKernelGGL(k_update_multidot<16>, dim3(nblk, nrhs), dim3(KB), 0, s, B, nv, h, hstride,
                       w, wstride, n, part, nblk, (int)always, need);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// w -= sum_i h[r*hstride + i] V_i
__global__ __launch_bounds__(KB) void k_update(Basis B, int nv, const double* __restrict__ h,
                                               int hstride, double* __restrict__ w,
                                               long long wstride, long long n) {
  const int r = blockIdx.y;
  const double* Vr = B.V + (long long)r * B.rstride;
  const double* hr = h + (long long)r * hstride;
  double* wr = w + (long long)r * wstride;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB) {
    double a = wr[e];
    for (int i = 0; i < nv; ++i) a -= hr[i] * Vr[(long long)i * B.vstride + e];
    wr[e] = a;
  }
}

hipError_t launch_update(Basis B, int nv, const double* h, int hstride, double* w,
                         long long wstride, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_update, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, h, hstride, w, wstride, n);
  return hipGetLastError();
}

// vout = (w - sum_i h_i V_i) / sqrt(max(0, nrm2 - sum_i h_i^2)); zero if that
// norm is zero, with (h, nrm2) = the coefficients and |w|^2 of the last pass
// that ran: h2 where need[r] (or need == nullptr: the second pass always
// ran), else h1 (rows of hstride values, |w|^2 at index nv).  The norm of the
// new vector follows from the norm before this pass because V is
// orthonormal.  NVMAX > 0: the basis values of an element are all loaded
// before use (nv <= NVMAX); NVMAX = 0: any nv.  With stage (host memory the
// device can write), block (0, r) also copies row r of h1, h2 and need[r]
// there: h1 rows at stage, h2 rows at stage + nrhs * hstride, the flags
// after them (as doubles, 1 where the second pass ran).
template <int NVMAX>
__global__ __launch_bounds__(KB) void k_update_normalize(Basis B, int nv,
                                                         const double* __restrict__ h1,
                                                         const double* __restrict__ h2,
                                                         int hstride, const int* __restrict__ need,
                                                         const double* __restrict__ w,
                                                         long long wstride,
                                                         double* __restrict__ vout, long long n,
                                                         double* stage) {
  const int r = blockIdx.y;
  if (stage && blockIdx.x == 0) {
    const int nrhs = gridDim.y;
    const long long o = (long long)r * hstride;
    for (int i = threadIdx.x; i < hstride; i += KB) {
      stage[o + i] = h1[o + i];
      stage[(long long)nrhs * hstride + o + i] = h2[o + i];
    }
    if (threadIdx.x == 0)
      stage[2LL * nrhs * hstride + r] = (need == nullptr || need[r]) ? 1.0 : 0.0;
    __threadfence_system();
  }
  const double* Vr = B.V + (long long)r * B.rstride;
  const double* hr = ((need == nullptr || need[r]) ? h2 : h1) + (long long)r * hstride;
  const double* wr = w + (long long)r * wstride;
  double* vr = vout + (long long)r * B.rstride;
  double hh = 0.0;
  for (int i = 0; i < nv; ++i) hh += hr[i] * hr[i];
  const double q = hr[nv] - hh;
  const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  if constexpr (NVMAX > 0) {
    double hv[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) hv[i] = i < nv ? hr[i] : 0.0;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
         e += (long long)gridDim.x * KB) {
      double v[NVMAX];
#pragma unroll
      for (int i = 0; i < NVMAX; ++i) v[i] = i < nv ? Vr[(long long)i * B.vstride + e] : 0.0;
      double a = wr[e];
#pragma unroll
      for (int i = 0; i < NVMAX; ++i) a -= hv[i] * v[i];
      vr[e] = a * inv;
    }
  } else {
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
         e += (long long)gridDim.x * KB) {
      double a = wr[e];
      for (int i = 0; i < nv; ++i) a -= hr[i] * Vr[(long long)i * B.vstride + e];
      vr[e] = a * inv;
    }
  }
}

hipError_t launch_update_normalize(Basis B, int nv, const double* h1, const double* h2,
                                   int hstride, const int* need, const double* w,
                                   long long wstride, double* vout, long long n, int nrhs,
                                   hipStream_t s, double* stage) {
  if (nv <= 8)
    hipLaunchKernelGGL(k_update_normalize<8>, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, h1, h2,
                       hstride, need, w, wstride, vout, n, stage);
  else if (nv <= 16)
    hipLaunchKernelGGL(k_update_normalize<16>, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, h1, h2,
                       hstride, need, w, wstride, vout, n, stage);
  else
    hipLaunchKernelGGL(k_update_normalize<0>, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, h1, h2,
                       hstride, need, w, wstride, vout, n, stage);
  return hipGetLastError();
}

// ------------------------------------------- delayed reorthogonalisation ----
// Arnoldi with one global reduction per step (classical Gram-Schmidt with
// the second pass delayed to the next step, after the DCGS2 scheme of
// Swirydowicz et al. and Bielich et al.).  Step j holds the final
// orthonormal v_0..v_{j-1} and a lagged vector u_j (slot j: once
// orthogonalised, scaled by a Pythagorean norm estimate).  It applies the
// operator to u_j, then one reduction gives a = V^T u_j, |u_j|^2, c = V^T w,
// u_j . w and |w|^2; from these
//   r = |u_j - V a| (by Pythagoras), v_j = (u_j - V a) / r   (final),
//   column j-1 of H final:  s_{j-1} + rho_j a, and rho_j r below it,
//   B v_j = (w - V H a) / r, so the first-pass coefficients of column j are
//   s_j = (V_{j+1}^T w - t) / r with t = H a, and
//   u_{j+1} = (w - V_{j+1} (t + r s_j)) / (r rho_{j+1}),
//   rho_{j+1} = sqrt(|B v_j|^2 - |s_j|^2).
// Step 0 starts from the cycle's unnormalised starting vector u_0 (b or a
// residual, read in place): with no basis yet, r = |u_0| and v_0 = u_0 / r,
// so the cycle needs no separate norm and scaling before its first step
// (the host takes |u_0|^2 from the staging of step 0).
//
// Device state per right-hand side (doubles, stride dstride): H column-major
// [K][K + 1], s_{j-1} [K + 1], a [K], t + r s [K + 1], then r, 1 / (r rho),
// rho.  Host staging per right-hand side (stride sstride): the final column
// j - 1 (rows 0..j), at K + 1 the estimated column j (rows 0..j), then
// rho_{j+1}, |B v_j|, r and a breakdown flag.

constexpr int DC_GROUP = 16;  // basis vectors per pass of the dot products

// One pass over G basis vectors i .. i+G-1 (G exact, so every load is one
// the pass needs): acc[q] += v_{i+q} . u, acc[DC_GROUP + q] += v_{i+q} . w,
// and with `first` also u.u, u.w, w.w.  All G + 2 loads of an element are
// issued before the first product.
template <int G>
__device__ inline void dcgs_pass(const double* Vr, long long vstride, int i, const double* u,
                                 const double* wr, long long e0, long long stride, long long n,
                                 bool first, double (&acc)[2 * DC_GROUP], double& uu, double& uw,
                                 double& ww) {
  for (long long e = e0; e < n; e += stride) {
    const double ue = u[e], we = wr[e];
    double ve[G];
#pragma unroll
    for (int q = 0; q < G; ++q) ve[q] = Vr[(long long)(i + q) * vstride + e];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      acc[q] += ve[q] * ue;
      acc[DC_GROUP + q] += ve[q] * we;
    }
    if (first) {
      uu += ue * ue;
      uw += ue * we;
      ww += we * we;
    }
  }
}

// rows of step j's reduction per right-hand side: a_0..a_{j-1}, |u|^2,
// c_0..c_{j-1}, u . w, |w|^2.  u_0 (j = 0): u0 + r u0stride when u0 is
// given, else slot 0.
__global__ __launch_bounds__(KB, 4) void k_dcgs_dots(Basis B, int j, const double* __restrict__ u0,
                                                  long long u0stride,
                                                  const double* __restrict__ w,
                                                  long long wstride, long long n,
                                                  double* __restrict__ part, int nblk) {
  __shared__ double sh[2 * DC_GROUP][KB / WAVE];
  const int r = blockIdx.y, wave = threadIdx.x >> 6, tid = threadIdx.x;
  const double* Vr = B.V + (long long)r * B.rstride;
  const double* u = j == 0 && u0 ? u0 + (long long)r * u0stride : Vr + (long long)j * B.vstride;
  const double* wr = w + (long long)r * wstride;
  const int rows = 2 * j + 3;
  double* pr = part + (long long)r * rows * nblk;
  const long long stride = (long long)nblk * KB;
  const long long e0 = (long long)blockIdx.x * KB + tid;
  // u.u, u.w, w.w ride along the first group's pass (a separate pass when
  // there is no basis vector yet)
  double uu = 0.0, uw = 0.0, ww = 0.0;
  for (int i = 0; i < j; i += DC_GROUP) {
    const int g = j - i < DC_GROUP ? j - i : DC_GROUP;  // block-uniform
    double acc[2 * DC_GROUP];
#pragma unroll
    for (int q = 0; q < 2 * DC_GROUP; ++q) acc[q] = 0.0;
    const bool first = i == 0;
    switch (g) {
#define R1S_PASS(G_) \
  case G_: dcgs_pass<G_>(Vr, B.vstride, i, u, wr, e0, stride, n, first, acc, uu, uw, ww); break;
      R1S_PASS(1) R1S_PASS(2) R1S_PASS(3) R1S_PASS(4) R1S_PASS(5) R1S_PASS(6) R1S_PASS(7)
      R1S_PASS(8) R1S_PASS(9) R1S_PASS(10) R1S_PASS(11) R1S_PASS(12) R1S_PASS(13)
      R1S_PASS(14) R1S_PASS(15) R1S_PASS(16)
#undef R1S_PASS
      default: break;
    }
    // block sums: value q < DC_GROUP is a_{i+q} (row i + q), value
    // DC_GROUP + q is c_{i+q} (row j + 1 + i + q)
#pragma unroll
    for (int q = 0; q < 2 * DC_GROUP; ++q) {
      if (q % DC_GROUP < g) {
        const double t = wave_sum(acc[q]);
        if (lane_id() == 0) sh[q][wave] = t;
      }
    }
    __syncthreads();
    if (tid < 2 * DC_GROUP && tid % DC_GROUP < g) {
      double t = 0.0;
      for (int w2 = 0; w2 < KB / WAVE; ++w2) t += sh[tid][w2];
      const int row = tid < DC_GROUP ? i + tid : j + 1 + i + (tid - DC_GROUP);
      pr[(long long)row * nblk + blockIdx.x] = t;
    }
    __syncthreads();
  }
  if (j == 0) {
    for (long long e = e0; e < n; e += stride) {
      const double ue = u[e], we = wr[e];
      uu += ue * ue;
      uw += ue * we;
      ww += we * we;
    }
  }
  uu = wave_sum(uu);
  uw = wave_sum(uw);
  ww = wave_sum(ww);
  if (lane_id() == 0) {
    sh[0][wave] = uu;
    sh[1][wave] = uw;
    sh[2][wave] = ww;
  }
  __syncthreads();
  if (tid < 3) {
    double t = 0.0;
    for (int w2 = 0; w2 < KB / WAVE; ++w2) t += sh[tid][w2];
    const int row = tid == 0 ? j : tid == 1 ? 2 * j + 1 : 2 * j + 2;
    pr[(long long)row * nblk + blockIdx.x] = t;
  }
}

hipError_t launch_dcgs_dots(Basis B, int j, const double* u0, long long u0stride, const double* w,
                            long long wstride, long long n, int nrhs, double* part, int nblk,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_dots, dim3(nblk, nrhs), dim3(KB), 0, s, B, j, u0, u0stride, w, wstride,
                     n, part, nblk);
  return hipGetLastError();
}

// One block per right-hand side: the fixed-order reduction of step j's rows
// (as k_reduce), then the small dense algebra spread over the block's
// threads (one thread per row of a column, sums by fixed-order block
// reductions): r, the final column j - 1, t = H a, s_j, rho_{j+1} and the
// update coefficients, staged for the host.  final_only: only r and the
// final column j - 1 (a cycle's last column).
__device__ inline void block_sum3(double& x, double& y, double& z, double (*sh)[KB / WAVE]) {
  x = wave_sum(x);
  y = wave_sum(y);
  z = wave_sum(z);
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sh[0][wave] = x;
    sh[1][wave] = y;
    sh[2][wave] = z;
  }
  __syncthreads();
  x = y = z = 0.0;
  for (int w = 0; w < KB / WAVE; ++w) {
    x += sh[0][w];
    y += sh[1][w];
    z += sh[2][w];
  }
  __syncthreads();
}

// Raises flag[r] = seq once the block's staging writes are visible to the
// host (each thread fenced at system scope before the barrier); the host
// spins on the flags instead of waiting for an event.
__device__ inline void stage_ready(int* flag, int r, int seq) {
  __syncthreads();
  if (flag && threadIdx.x == 0)
    __hip_atomic_store(flag + r, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(KB) void k_dcgs_small(int j, int K, const double* __restrict__ part,
                                                   int nblk, double* __restrict__ dstate,
                                                   long long dstride, double* stage, int sstride,
                                                   int final_only, int* flag, int seq) {
  extern __shared__ double red[];  // the 2j + 3 sums, then t [j + 1]
  __shared__ double bs[3][KB / WAVE];
  const int r = blockIdx.x, rows = 2 * j + 3, tid = threadIdx.x;
  const double* pr = part + (long long)r * rows * nblk;
  for (int row = tid >> 6; row < rows; row += KB / WAVE) {
    double v[REDUCE_PER_LANE];
#pragma unroll
    for (int t = 0; t < REDUCE_PER_LANE; ++t) {
      const int b = lane_id() + t * WAVE;
      v[t] = b < nblk ? pr[(long long)row * nblk + b] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < REDUCE_PER_LANE; ++t) a += v[t];
    a = wave_sum(a);
    if (lane_id() == 0) red[row] = a;
  }
  __syncthreads();
  double* H = dstate + (long long)r * dstride;
  double* sprev = H + (long long)K * (K + 1);
  double* aco = sprev + (K + 1);
  double* gco = aco + K;
  double* sc = gco + (K + 1);
  double* st = stage + (long long)r * sstride;
  const double* a = red;
  const double alpha = red[j];
  const double* c = red + j + 1;
  const double gam = red[2 * j + 1], om = red[2 * j + 2];
  double* tsh = red + rows;
  // |a|^2 and a . c
  double aa = 0.0, ac = 0.0, dummy = 0.0;
  for (int i = tid; i < j; i += KB) {
    aa += a[i] * a[i];
    ac += a[i] * c[i];
  }
  block_sum3(aa, ac, dummy, bs);
  const double r2 = alpha - aa;
  const bool brk = !(r2 > 0.0);
  const double rr = brk ? 1.0 : sqrt(r2);
  if (j == 0 && tid == 0) st[0] = alpha;  // |u_0|^2 (no final column at step 0)
  if (j > 0) {
    const double rho_prev = sc[2];
    double* col = H + (long long)(j - 1) * (K + 1);
    for (int i = tid; i <= j; i += KB) {
      const double h = i < j ? sprev[i] + rho_prev * a[i] : rho_prev * rr;
      col[i] = h;
      st[i] = h;
    }
  }
  for (int i = tid; i < j; i += KB) aco[i] = a[i];
  if (tid == 0) sc[0] = rr;
  if (final_only) {
    if (tid == 0) {
      st[2 * K + 4] = rr;
      st[2 * K + 5] = brk ? 1.0 : 0.0;
    }
    __threadfence_system();
    stage_ready(flag, r, seq);
    return;
  }
  __syncthreads();  // column j - 1 of H written before it is read below
  // t_i = sum_l H[l][i] a_l over the columns l >= i - 1 (column l has rows 0..l+1)
  for (int i = tid; i <= j; i += KB) {
    // four independent partial sums so that their loads overlap, added in a
    // fixed order
    double t4[4] = {0.0, 0.0, 0.0, 0.0};
    int l = i > 0 ? i - 1 : 0;
    for (; l + 4 <= j; l += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) t4[q] += H[(long long)(l + q) * (K + 1) + i] * a[l + q];
    }
    for (; l < j; ++l) t4[0] += H[(long long)l * (K + 1) + i] * a[l];
    tsh[i] = (t4[0] + t4[1]) + (t4[2] + t4[3]);
  }
  __syncthreads();
  // d = V_{j+1}^T w, s = (d - t) / r, g = t + r s; |B v_j|^2 from t.d, |t|^2
  const double inv_r = 1.0 / rr;
  double td = 0.0, tt = 0.0, ss = 0.0;
  for (int i = tid; i <= j; i += KB) {
    const double di = i < j ? c[i] : (gam - ac) * inv_r;
    const double ti = tsh[i];
    const double si = (di - ti) * inv_r;
    td += ti * di;
    tt += ti * ti;
    ss += si * si;
    sprev[i] = si;
    st[K + 1 + i] = si;
    gco[i] = ti + rr * si;
  }
  block_sum3(td, tt, ss, bs);
  if (tid == 0) {
    const double nw2 = (om - 2.0 * td + tt) * inv_r * inv_r;
    const double q = nw2 - ss;
    const double rho = q > 0.0 ? sqrt(q) : 0.0;
    sc[1] = rho > 0.0 ? 1.0 / (rr * rho) : 0.0;
    sc[2] = rho;
    st[2 * K + 2] = rho;
    st[2 * K + 3] = nw2 > 0.0 ? sqrt(nw2) : 0.0;
    st[2 * K + 4] = rr;
    st[2 * K + 5] = brk ? 1.0 : 0.0;
  }
  __threadfence_system();
  stage_ready(flag, r, seq);
}

hipError_t launch_dcgs_small(int j, int K, const double* part, int nblk, double* dstate,
                             long long dstride, double* stage, int sstride, bool final_only,
                             int nrhs, hipStream_t s, int* flag, int seq) {
  if (nblk > REDUCE_PER_LANE * WAVE) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dcgs_small, dim3(nrhs), dim3(KB), (size_t)(3 * j + 4) * sizeof(double), s,
                     j, K, part, nblk, dstate, dstride, stage, sstride, (int)final_only, flag,
                     seq);
  return hipGetLastError();
}

// flag[0] = seq after everything before it on the stream (a device-to-host
// copy into pinned memory, say) has completed.
__global__ void k_stage_flag(int* flag, int seq) {
  __threadfence_system();
  __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_stage_flag(int* flag, int seq, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_flag, dim3(1), dim3(1), 0, s, flag, seq);
  return hipGetLastError();
}

// v_j = (u_j - V a) / r in slot j and u_{j+1} = (w - V_{j+1} g) / (r rho)
// in slot j + 1, g = t + r s (device state of k_dcgs_small); u_0 as in
// k_dcgs_dots.
__global__ __launch_bounds__(KB) void k_dcgs_update(Basis B, int j, int K,
                                                    const double* __restrict__ dstate,
                                                    long long dstride, const double* u0,
                                                    long long u0stride, const double* __restrict__ w,
                                                    long long wstride, long long n) {
  const int r = blockIdx.y;
  double* Vr = B.V + (long long)r * B.rstride;
  const double* ur = j == 0 && u0 ? u0 + (long long)r * u0stride : Vr + (long long)j * B.vstride;
  const double* wr = w + (long long)r * wstride;
  const double* sprev = dstate + (long long)r * dstride + (long long)K * (K + 1);
  const double* aco = sprev + (K + 1);
  const double* gco = aco + K;
  const double* sc = gco + (K + 1);
  const double inv_r = 1.0 / sc[0], inv2 = sc[1], gj = gco[j];
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB) {
    const double uj = ur[e];
    double av = uj, au = wr[e];
    for (int i = 0; i < j; ++i) {
      const double vi = Vr[(long long)i * B.vstride + e];
      av -= aco[i] * vi;
      au -= gco[i] * vi;
    }
    const double vj = av * inv_r;
    Vr[(long long)j * B.vstride + e] = vj;
    Vr[(long long)(j + 1) * B.vstride + e] = (au - gj * vj) * inv2;
  }
}

hipError_t launch_dcgs_update(Basis B, int j, int K, const double* dstate, long long dstride,
                              const double* u0, long long u0stride, const double* w,
                              long long wstride, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_update, vec_grid(n, nrhs), dim3(KB), 0, s, B, j, K, dstate, dstride,
                     u0, u0stride, w, wstride, n);
  return hipGetLastError();
}

// out_r = w_r * inv[r]
__global__ __launch_bounds__(KB) void k_scale(const double* __restrict__ w, long long wstride,
                                              const double* __restrict__ inv,
                                              double* __restrict__ out, long long ostride,
                                              long long n) {
  const int r = blockIdx.y;
  const double s = inv[r];
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB)
    out[(long long)r * ostride + e] = w[(long long)r * wstride + e] * s;
}

hipError_t launch_scale(const double* w, long long wstride, const double* inv, double* out,
                        long long ostride, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, vec_grid(n, nrhs), dim3(KB), 0, s, w, wstride, inv, out, ostride, n);
  return hipGetLastError();
}

// out_r = w_r / |w_r| from the squared norms sq[r] (0 where |w_r| = 0)
__global__ __launch_bounds__(KB) void k_scale_unit(const double* __restrict__ w, long long wstride,
                                                   const double* __restrict__ sq,
                                                   double* __restrict__ out, long long ostride,
                                                   long long n) {
  const int r = blockIdx.y;
  const double q = sq[r];
  const double s = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB)
    out[(long long)r * ostride + e] = w[(long long)r * wstride + e] * s;
}

hipError_t launch_scale_unit(const double* w, long long wstride, const double* sq, double* out,
                             long long ostride, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_unit, vec_grid(n, nrhs), dim3(KB), 0, s, w, wstride, sq, out, ostride,
                     n);
  return hipGetLastError();
}

// out_r = sum_i y[r*ystride + i] V_i
__global__ __launch_bounds__(KB) void k_combine(Basis B, int nv, const double* __restrict__ y,
                                                int ystride, double* __restrict__ out,
                                                long long ostride, long long n) {
  const int r = blockIdx.y;
  const double* Vr = B.V + (long long)r * B.rstride;
  const double* yr = y + (long long)r * ystride;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB) {
    double a = 0.0;
    for (int i = 0; i < nv; ++i) a += yr[i] * Vr[(long long)i * B.vstride + e];
    out[(long long)r * ostride + e] = a;
  }
}

hipError_t launch_combine(Basis B, int nv, const double* y, int ystride, double* out,
                          long long ostride, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, y, ystride, out, ostride,
                     n);
  return hipGetLastError();
}

// k_combine with the coefficients passed by value (y[r * nv + i]): no copy
// of y to the device before the launch
__global__ __launch_bounds__(KB) void k_combine_arg(Basis B, int nv, CombineY y,
                                                    double* __restrict__ out, long long ostride,
                                                    long long n) {
  const int r = blockIdx.y;
  const double* Vr = B.V + (long long)r * B.rstride;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB) {
    double a = 0.0;
    for (int i = 0; i < nv; ++i) a += y.y[r * nv + i] * Vr[(long long)i * B.vstride + e];
    out[(long long)r * ostride + e] = a;
  }
}

hipError_t launch_combine_arg(Basis B, int nv, const double* y, int ystride, double* out,
                              long long ostride, long long n, int nrhs, hipStream_t s) {
  if ((long long)nrhs * nv > COMBINE_Y_MAX) return hipErrorInvalidValue;
  CombineY ya;
  for (int r = 0; r < nrhs; ++r)
    for (int i = 0; i < nv; ++i) ya.y[r * nv + i] = y[(size_t)r * ystride + i];
  hipLaunchKernelGGL(k_combine_arg, vec_grid(n, nrhs), dim3(KB), 0, s, B, nv, ya, out, ostride,
                     n);
  return hipGetLastError();
}

// y_r += alpha[r] x_r  (alpha == nullptr: 1); contiguous [nrhs][n]
__global__ __launch_bounds__(KB) void k_axpy(const double* __restrict__ alpha,
                                             const double* __restrict__ xv,
                                             double* __restrict__ yv, long long n) {
  const int r = blockIdx.y;
  const double a = alpha ? alpha[r] : 1.0;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB)
    yv[(long long)r * n + e] += a * xv[(long long)r * n + e];
}

hipError_t launch_axpy(const double* alpha, const double* xv, double* yv, long long n, int nrhs,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, vec_grid(n, nrhs), dim3(KB), 0, s, alpha, xv, yv, n);
  return hipGetLastError();
}

// y_r = b_r - y_r ; contiguous [nrhs][n]
__global__ __launch_bounds__(KB) void k_rsub(const double* __restrict__ bv,
                                             double* __restrict__ yv, long long n) {
  const int r = blockIdx.y;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n;
       e += (long long)gridDim.x * KB)
    yv[(long long)r * n + e] = bv[(long long)r * n + e] - yv[(long long)r * n + e];
}

hipError_t launch_rsub(const double* bv, double* yv, long long n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_rsub, vec_grid(n, nrhs), dim3(KB), 0, s, bv, yv, n);
  return hipGetLastError();
}

}  // namespace r1s
