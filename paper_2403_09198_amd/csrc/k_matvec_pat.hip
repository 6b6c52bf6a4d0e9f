// Matvec instantiations for a general pattern of the diagonal block (any
// pair counts), in a file of their own so that the library's kernels compile
// in parallel.
#include "k_matvec_impl.hpp"

namespace r1s {

template <typename TV, bool TRANS, bool RESID>
static hipError_t mv_pat(const Mesh& g, const TV* rec, const double* x, const double* b,
                         double* y, int nrhs, hipStream_t s) {
  if (g.ro <= RANK_OFF_SMALL)
    return launch_mv_r<TV, TRANS, RESID, RANK_DIAG_MAX, RANK_OFF_SMALL, 2>(g, rec, x, b, y, nrhs, s);
  return launch_mv_r<TV, TRANS, RESID, RANK_DIAG_MAX, RANK_OFF_MAX, 2>(g, rec, x, b, y, nrhs, s);
}

// kind: bit 0 transpose, bit 1 residual (float64 only), bit 2 float32 values
hipError_t launch_mv_pattern(const Mesh& g, const void* rec, int kind, const double* x,
                             const double* b, double* y, int nrhs, hipStream_t s) {
  const double* r64 = (const double*)rec;
  const float* r32 = (const float*)rec;
  switch (kind) {
    case 0: return mv_pat<double, false, false>(g, r64, x, b, y, nrhs, s);
    case 1: return mv_pat<double, true, false>(g, r64, x, b, y, nrhs, s);
    case 2: return mv_pat<double, false, true>(g, r64, x, b, y, nrhs, s);
    case 3: return mv_pat<double, true, true>(g, r64, x, b, y, nrhs, s);
    case 4: return mv_pat<float, false, false>(g, r32, x, b, y, nrhs, s);
    case 5: return mv_pat<float, true, false>(g, r32, x, b, y, nrhs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace r1s
