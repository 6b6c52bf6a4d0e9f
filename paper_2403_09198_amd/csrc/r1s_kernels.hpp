// Host-callable kernel launchers of libr1s (all asynchronous on `s`).
#pragma once
#include <hip/hip_runtime.h>

#include "r1s_device.hpp"

namespace r1s {

struct PackIn {
  const double *s_diag, *s_sub, *s_sup, *s_flow, *s_nbr, *u, *v;
  const double *s_band, *s_lev_flow, *s_flow_lev;  // wide diagonal-block pattern only
  const double* s_cc;  // general pattern: [N][nnz] (the structured S_cc arrays unused)
};

// inputs on a general mesh (per cell: diagonal block; per off-diagonal block
// in input order: its diagonal and pairs)
struct GraphPackIn {
  const double *s_diag, *s_sub, *s_sup, *s_flow, *s_band, *s_lev_flow, *s_flow_lev;
  const double *s_nbr, *u_diag, *v_diag, *u_off, *v_off;
};

struct GraphGradOut {
  double *s_diag, *s_sub, *s_sup, *s_flow, *s_band, *s_lev_flow, *s_flow_lev;
  double *s_nbr, *u_diag, *v_diag, *u_off, *v_off;
};

struct GradOut {
  double *s_diag, *s_sub, *s_sup, *s_flow, *s_nbr, *u, *v;
  double *s_band, *s_lev_flow, *s_flow_lev;
  double* s_cc;  // general pattern: [N][nnz] (the structured S_cc outputs unused)
};

// pair counts the kernels are built for
bool ranks_supported(int rd, int ro);

// packing / casting
hipError_t launch_pack(const Mesh& g, const PackIn& in, double* rec64, float* rec32, hipStream_t s);
hipError_t launch_cast_f32(const double* src, float* dst, long long count, hipStream_t s);

// general mesh: packing, matvec / residual, gradients
hipError_t launch_pack_graph(const Mesh& g, const GraphPackIn& in, double* rec64, float* rec32,
                             hipStream_t s);
hipError_t launch_matvec_graph(const Mesh& g, const void* rec, bool f32, bool trans,
                               const double* x, const double* b, double* y, int nrhs, bool resid,
                               hipStream_t s);
hipError_t launch_grad_graph(const Mesh& g, const double* rec, const double* lam, const double* x,
                             int nrhs, const GraphGradOut& out, hipStream_t s);

// structured matvec, general-rank instantiations (kind: bit 0 transpose,
// bit 1 residual, bit 2 float32 values); ro <= 2 and ro <= 6
hipError_t launch_mv_general_r2(const Mesh& g, const void* rec, int kind, const double* x,
                                const double* b, double* y, int nrhs, hipStream_t s);
hipError_t launch_mv_general_r6(const Mesh& g, const void* rec, int kind, const double* x,
                                const double* b, double* y, int nrhs, hipStream_t s);
// the same for a general pattern of the diagonal block
hipError_t launch_mv_pattern(const Mesh& g, const void* rec, int kind, const double* x,
                             const double* b, double* y, int nrhs, hipStream_t s);

// structured matvec (rec: packed record, float when f32)
hipError_t launch_matvec(const Mesh& g, const void* rec, bool f32, bool trans, const double* x,
                         double* y, int nrhs, hipStream_t s);
hipError_t launch_residual(const Mesh& g, const double* rec, bool trans, const double* b,
                           const double* x, double* r, int nrhs, hipStream_t s);

// Packed workgroup forms (one pair per block, tridiagonal band, no
// coupling, one right-hand side r0 per launch): y = J x / J^T x / b - J x
// for 32 <= m <= 256 (packed_ok), and z = M r / M^T r for 32 <= m < 64
// (packed_apply_ok)
bool packed_ok(const Mesh& g);
bool packed_apply_ok(const Mesh& g);
hipError_t launch_matvec_packed(const Mesh& g, const void* rec, bool f32, bool trans, bool resid,
                                const double* x, const double* b, double* y, int r0,
                                hipStream_t s);
hipError_t launch_smw_apply_packed(const Mesh& g, const void* fac, const void* invC, bool f32,
                                   bool trans, const double* r, double* z, int r0,
                                   hipStream_t s);

// SMW block-Jacobi
// invC: per cell the rd x rd inverse capacitance matrix, forward then (when
// facT) transposed, [2][N][rd][rd] (one [N][rd][rd] without facT)
hipError_t launch_smw_setup(const Mesh& g, const double* rec, double* facF, double* facT,
                            double* invC, int* status, hipStream_t s);
hipError_t launch_smw_apply(const Mesh& g, const void* fac, const void* invC, bool f32, bool trans,
                            const double* r, double* z, int nrhs, hipStream_t s);
hipError_t launch_fill_int(int* p, int value, int count, hipStream_t s);
// y = J x and z = M y in one kernel (one right-hand side, forward); only
// where matvec_prec_fused(g, f32) holds (else hipErrorInvalidValue)
bool matvec_prec_fused(const Mesh& g, bool f32);
hipError_t launch_matvec_prec(const Mesh& g, const void* rec, const void* fac, const void* invC,
                              bool f32, const double* x, double* y, double* z, hipStream_t s);

// SMW block-Jacobi for the wide diagonal-block pattern (band > 1 or level/flow
// coupling): tile-interleaved factors, 32 cells per tile.  wvT may be null.
void band_prec_counts(const Mesh& g, long long* bf, long long* s3i, long long* wv,
                      long long* cinv);
hipError_t launch_band_setup(const Mesh& g, const double* rec, double* bf, double* s3i,
                             double* wv, double* wvT, double* cinv, int* status, hipStream_t s);
hipError_t launch_band_apply(const Mesh& g, const void* bf, const void* s3i, const void* wv,
                             const void* cinv, bool f32, bool trans, const double* r, double* z,
                             int nrhs, hipStream_t s);
// The same for a general pattern: LU of the permuted S_cc with the fill of
// the plan (factor positions lu.nnzF per cell, tile-interleaved), then the
// Woodbury correction as above.
void pattern_prec_counts(const Mesh& g, int nnzF, long long* bf, long long* wv, long long* cinv);
hipError_t launch_pattern_setup(const Mesh& g, const PatLU& lu, const double* rec, double* bf,
                                double* wv, double* wvT, double* cinv, int* status, hipStream_t s);
hipError_t launch_pattern_apply(const Mesh& g, const PatLU& lu, const void* bf, const void* wv,
                                const void* cinv, bool f32, bool trans, const double* r,
                                double* z, int nrhs, hipStream_t s);

// dense-block BSR baseline
hipError_t launch_bsr_assemble(const Mesh& g, const double* rec, const int* blk_row,
                               const int* blk_dir, long long nblocks, double* data, hipStream_t s);
hipError_t launch_bsr_matvec(const Mesh& g, const int* indptr, const int* indices,
                             const double* data, const double* x, double* y, int nrhs,
                             hipStream_t s);
hipError_t launch_bsr_lu_setup(const Mesh& g, const int* diag_block, const double* data,
                               double* lu, int* piv, int* status, hipStream_t s);
bool bsr_lu_fits_lds(const Mesh& g);
hipError_t launch_bsr_gather_diag(const Mesh& g, const int* diag_block, const double* data,
                                  double* lu, hipStream_t s);
hipError_t launch_bsr_piv_convert(const Mesh& g, int* piv, const int* info, int* status,
                                  hipStream_t s);
hipError_t launch_bsr_lu_apply(const Mesh& g, const double* lu, const int* piv, const double* r,
                               double* z, int nrhs, hipStream_t s);

// Krylov vector kernels (float64).  Vectors of length n per right-hand
// side; V holds nv basis vectors per right-hand side with stride vstride
// between vectors and rstride between right-hand sides.
struct Basis {
  double* V;
  long long vstride, rstride;
};
int dot_blocks(long long n);
hipError_t launch_multidot(Basis B, int nv, const double* w, long long wstride, long long n,
                           int nrhs, double* part, int nblk, bool with_norm, hipStream_t s);
hipError_t launch_reduce(const double* part, int rows, int nblk, double* out, hipStream_t s);
// the same in one workgroup, also writing host[row] (pinned) and then
// flag[0] = seq (see launch_stage_flag)
hipError_t launch_reduce_host(const double* part, int rows, int nblk, double* out, double* host,
                              int* flag, int seq, hipStream_t s);
int update_multidot_max();
hipError_t launch_update_multidot(Basis B, int nv, const double* h, int hstride, double* w,
                                  long long wstride, long long n, int nrhs, double* part, int nblk,
                                  bool always, int* need, hipStream_t s);
hipError_t launch_update(Basis B, int nv, const double* h, int hstride, double* w,
                         long long wstride, long long n, int nrhs, hipStream_t s);
// Delayed reorthogonalisation (one reduction per Arnoldi step; k_krylov.hip)
// u0 (or null: slot 0): the unnormalised starting vector of step 0, per
// right-hand side at u0 + r u0stride
hipError_t launch_dcgs_dots(Basis B, int j, const double* u0, long long u0stride, const double* w,
                            long long wstride, long long n, int nrhs, double* part, int nblk,
                            hipStream_t s);
// flag (pinned host memory, or null): flag[r] = seq once right-hand side r's
// staging is visible to the host
hipError_t launch_dcgs_small(int j, int K, const double* part, int nblk, double* dstate,
                             long long dstride, double* stage, int sstride, bool final_only,
                             int nrhs, hipStream_t s, int* flag = nullptr, int seq = 0);
// flag[0] = seq once the stream's earlier work has completed
hipError_t launch_stage_flag(int* flag, int seq, hipStream_t s);
hipError_t launch_dcgs_update(Basis B, int j, int K, const double* dstate, long long dstride,
                              const double* u0, long long u0stride, const double* w,
                              long long wstride, long long n, int nrhs, hipStream_t s);
hipError_t launch_update_normalize(Basis B, int nv, const double* h1, const double* h2,
                                   int hstride, const int* need, const double* w,
                                   long long wstride, double* vout, long long n, int nrhs,
                                   hipStream_t s, double* stage = nullptr);
hipError_t launch_scale(const double* w, long long wstride, const double* inv, double* out,
                        long long ostride, long long n, int nrhs, hipStream_t s);
hipError_t launch_scale_unit(const double* w, long long wstride, const double* sq, double* out,
                             long long ostride, long long n, int nrhs, hipStream_t s);
hipError_t launch_combine(Basis B, int nv, const double* y, int ystride, double* out,
                          long long ostride, long long n, int nrhs, hipStream_t s);
// the same with y in host memory passed by value (nrhs * nv <= COMBINE_Y_MAX)
constexpr int COMBINE_Y_MAX = 64;
struct CombineY {
  double y[COMBINE_Y_MAX];
};
hipError_t launch_combine_arg(Basis B, int nv, const double* y, int ystride, double* out,
                              long long ostride, long long n, int nrhs, hipStream_t s);
hipError_t launch_rsub(const double* bv, double* yv, long long n, int nrhs, hipStream_t s);
hipError_t launch_axpy(const double* alpha, const double* xv, double* yv, long long n, int nrhs,
                       hipStream_t s);

// gradients
hipError_t launch_grad(const Mesh& g, const double* rec, const double* lam, const double* x,
                       int nrhs, const GradOut& out, hipStream_t s);

}  // namespace r1s
