// Launchers of the packed workgroup kernels (k_packed_impl.hpp) and the
// choice of their workgroup size.
//
// Measured on MI355X (512 x 256 mesh, float64, non-temporal output stores,
// cache flushed before each launch; algorithmic bytes / kernel time):
//
//   m    matvec: packed (waves)   wave per chunk    SMW apply: packed   wave per cell
//   35   127 us (4) 0.68          164 us 0.53       54.7 us (4) 0.58    64.2 us 0.50
//        (unpadded rows; 8 or 16 waves: 131 us)
//   64   205 us (4) 0.78          216 us 0.73       78.9 us (4) 0.74    78.3 us 0.75
//   123  414 us (8) 0.74          430 us 0.71       156 us (2)  0.72    workgroup 147-159 us
//   203  688 us (16) 0.73         767 us 0.66       318 us (16) 0.59    249 us 0.75
//
// Consecutive-cell (plain) tiles beat column-band tiles in every case,
// although the band map halves the L2 misses of the neighbour x blocks.
#include "k_packed_impl.hpp"

namespace r1s {

bool packed_ok(const Mesh& g) {
  return !g.graph && g.rd == 1 && g.ro == 1 && !wide_pattern(g) && g.m >= PK_MMIN &&
         g.m <= MAX_CHUNKS * WAVE;
}

bool packed_apply_ok(const Mesh& g) { return packed_ok(g) && g.m < WAVE; }

// Waves per matvec workgroup: the fewest of 4, 8, 16 that keep 95% of the
// lanes busy (m = 35: 4 waves hold 7 cells in 245 of 256 lanes; m = 203: 16
// waves hold 5 cells in 1015 of 1024), else the best-filled.
static int packed_nw(int m) {
  int best = 4;
  double best_fill = 0.0;
  for (int nw : {4, 8, 16}) {
    const int t = nw * WAVE;
    const double fill = (double)(t / m) * m / t;
    if (fill >= 0.95) return nw;
    if (fill > best_fill + 1e-9) {
      best_fill = fill;
      best = nw;
    }
  }
  return best;
}

template <typename TV, int NW, bool TRANS, bool RESID>
static hipError_t launch_mv_pk_nw(const Mesh& g, const TV* rec, const double* x,
                                  const double* b, double* y, int r0, hipStream_t s) {
  const int Q = NW * WAVE / g.m;
  const int grid = cell_grid<false>(g, Q);
  if (g.m >= WAVE)
    hipLaunchKernelGGL((k_matvec_pk<TV, NW, 2, TRANS, RESID, false>), dim3(grid),
                       dim3(NW * WAVE), 0, s, g, rec, x, b, y, Q, r0);
  else
    hipLaunchKernelGGL((k_matvec_pk<TV, NW, 3, TRANS, RESID, false>), dim3(grid),
                       dim3(NW * WAVE), 0, s, g, rec, x, b, y, Q, r0);
  return hipGetLastError();
}

template <typename TV, bool TRANS, bool RESID>
static hipError_t launch_mv_pk_t(const Mesh& g, const TV* rec, const double* x, const double* b,
                                 double* y, int r0, hipStream_t s) {
  switch (packed_nw(g.m)) {
    case 4: return launch_mv_pk_nw<TV, 4, TRANS, RESID>(g, rec, x, b, y, r0, s);
    case 8: return launch_mv_pk_nw<TV, 8, TRANS, RESID>(g, rec, x, b, y, r0, s);
    default: return launch_mv_pk_nw<TV, 16, TRANS, RESID>(g, rec, x, b, y, r0, s);
  }
}

hipError_t launch_matvec_packed(const Mesh& g, const void* rec, bool f32, bool trans,
                                bool resid, const double* x, const double* b, double* y, int r0,
                                hipStream_t s) {
  if (!packed_ok(g) || (resid && f32)) return hipErrorInvalidValue;
  if (f32) {
    const float* r = (const float*)rec;
    return trans ? launch_mv_pk_t<float, true, false>(g, r, x, b, y, r0, s)
                 : launch_mv_pk_t<float, false, false>(g, r, x, b, y, r0, s);
  }
  const double* r = (const double*)rec;
  if (resid)
    return trans ? launch_mv_pk_t<double, true, true>(g, r, x, b, y, r0, s)
                 : launch_mv_pk_t<double, false, true>(g, r, x, b, y, r0, s);
  return trans ? launch_mv_pk_t<double, true, false>(g, r, x, b, y, r0, s)
               : launch_mv_pk_t<double, false, false>(g, r, x, b, y, r0, s);
}

// SMW apply, m < 64: four waves (seven cells at m = 35).
template <typename TV, bool TRANS>
static hipError_t launch_apply_pk_t(const Mesh& g, const TV* fac, const TV* invC, const double* r,
                                    double* z, int r0, hipStream_t s) {
  constexpr int NW = 4;
  const int Q = NW * WAVE / g.m;
  const int grid = (g.N + Q - 1) / Q;
  hipLaunchKernelGGL((k_smw_apply_pk<TV, NW, 3, TRANS>), dim3(grid), dim3(NW * WAVE), 0, s, g,
                     fac, invC, r, z, Q, r0);
  return hipGetLastError();
}

hipError_t launch_smw_apply_packed(const Mesh& g, const void* fac, const void* invC, bool f32,
                                   bool trans, const double* r, double* z, int r0,
                                   hipStream_t s) {
  if (!packed_apply_ok(g)) return hipErrorInvalidValue;
  if (f32)
    return trans ? launch_apply_pk_t<float, true>(g, (const float*)fac, (const float*)invC, r, z, r0, s)
                 : launch_apply_pk_t<float, false>(g, (const float*)fac, (const float*)invC, r, z, r0, s);
  return trans ? launch_apply_pk_t<double, true>(g, (const double*)fac, (const double*)invC, r, z, r0, s)
               : launch_apply_pk_t<double, false>(g, (const double*)fac, (const double*)invC, r, z, r0, s);
}

}  // namespace r1s
