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
