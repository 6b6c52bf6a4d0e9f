/*
 * A plain C caller of libr1s (no Python, no torch): reads a small problem
 * from a binary file, runs the library's matvec, transposed matvec, SMW
 * block-Jacobi apply (and its transpose), the fused J x / M (J x) call and a
 * GMRES solve through the C ABI
 * of include/r1s.h with device memory from the HIP runtime, and writes the
 * results to a binary file for the parity test to compare with the oracle.
 *
 *   abi_client <in.bin> <out.bin>
 *
 * in.bin : int32 magic 0x31533152, nx, ny, L, r_diag, r_off; then float64
 *          s_diag [N][m], s_sub [N][L-1], s_sup [N][L-1], s_flow [N][6],
 *          s_nbr [N][4][m], u [N][P][m], v [N][P][m], x [N][m], b [N][m]
 *          (tridiagonal level band, no level/flow coupling).
 * out.bin: float64 J x, J^T x, M x, M^T x, the GMRES solution of J x = b
 *          (rtol 1e-12), J x and M (J x) from r1s_matvec_prec, each [N][m];
 *          then int32 iterations, converged.
 * Exit status 0 on success; on failure the library's message goes to stderr.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "r1s.h"

#define CHECK_HIP(call)                                                    \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));           \
      return 2;                                                            \
    }                                                                      \
  } while (0)

#define CHECK_R1S(call)                                                    \
  do {                                                                     \
    int e_ = (call);                                                       \
    if (e_ != R1S_OK) {                                                    \
      fprintf(stderr, "%s: %d (%s)\n", #call, e_, r1s_last_error());       \
      return 3;                                                            \
    }                                                                      \
  } while (0)

static int read_all(FILE* f, void* p, size_t bytes) {
  return fread(p, 1, bytes, f) == bytes ? 0 : -1;
}

/* Host array of `count` float64 read from f, copied to a new device buffer. */
static int load_dev(FILE* f, size_t count, double** dev) {
  double* h = (double*)malloc(count * sizeof(double) + 8);
  if (!h || read_all(f, h, count * sizeof(double))) {
    free(h);
    fprintf(stderr, "short input file\n");
    return 1;
  }
  *dev = NULL;
  if (count > 0) {
    if (hipMalloc((void**)dev, count * sizeof(double)) != hipSuccess ||
        hipMemcpy(*dev, h, count * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      free(h);
      fprintf(stderr, "device copy failed\n");
      return 2;
    }
  }
  free(h);
  return 0;
}

static int save_dev(FILE* f, const double* dev, size_t count) {
  double* h = (double*)malloc(count * sizeof(double));
  if (!h) return 1;
  if (hipMemcpy(h, dev, count * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      fwrite(h, sizeof(double), count, f) != count) {
    free(h);
    return 2;
  }
  free(h);
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <in.bin> <out.bin>\n", argv[0]);
    return 1;
  }
  FILE* fi = fopen(argv[1], "rb");
  if (!fi) {
    perror(argv[1]);
    return 1;
  }
  int32_t hdr[6];
  if (read_all(fi, hdr, sizeof hdr) || hdr[0] != 0x31533152) {
    fprintf(stderr, "bad header\n");
    return 1;
  }
  const int nx = hdr[1], ny = hdr[2], L = hdr[3];
  const r1s_layout lay = {hdr[4], hdr[5], 1, 0};
  const size_t N = (size_t)nx * ny, m = (size_t)L + 3, P = (size_t)lay.r_diag + 4 * lay.r_off;
  const size_t n = N * m;

  double *s_diag, *s_sub, *s_sup, *s_flow, *s_nbr, *u, *v, *x, *b;
  if (load_dev(fi, N * m, &s_diag) || load_dev(fi, N * (L - 1), &s_sub) ||
      load_dev(fi, N * (L - 1), &s_sup) || load_dev(fi, N * 6, &s_flow) ||
      load_dev(fi, N * 4 * m, &s_nbr) || load_dev(fi, N * P * m, &u) ||
      load_dev(fi, N * P * m, &v) || load_dev(fi, n, &x) || load_dev(fi, n, &b))
    return 1;
  fclose(fi);

  /* matrix: the caller owns the device buffer */
  size_t bytes = 0;
  CHECK_R1S(r1s_mat_size(nx, ny, L, &lay, 0, &bytes));
  void* mat_mem = NULL;
  CHECK_HIP(hipMalloc(&mat_mem, bytes));
  const r1s_inputs in = {s_diag, L > 1 ? s_sub : NULL, L > 1 ? s_sup : NULL, s_flow, s_nbr,
                         u, v, NULL, NULL, NULL};
  r1s_mat A = NULL;
  CHECK_R1S(r1s_mat_init(nx, ny, L, &lay, 0, &in, mat_mem, bytes, NULL, &A));

  double *y, *yt, *z, *zt, *xs, *yf, *zf;
  CHECK_HIP(hipMalloc((void**)&y, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&yt, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&z, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&zt, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&xs, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&yf, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&zf, n * sizeof(double)));
  CHECK_R1S(r1s_matvec(A, R1S_F64, 0, 1, x, y, NULL));
  CHECK_R1S(r1s_matvec(A, R1S_F64, 1, 1, x, yt, NULL));

  /* block-Jacobi preconditioner with its transpose */
  CHECK_R1S(r1s_prec_size(A, R1S_WITH_TRANS, &bytes));
  void* prec_mem = NULL;
  CHECK_HIP(hipMalloc(&prec_mem, bytes));
  r1s_prec M = NULL;
  CHECK_R1S(r1s_prec_setup(A, R1S_WITH_TRANS, prec_mem, bytes, NULL, &M));
  CHECK_R1S(r1s_prec_apply(M, R1S_F64, 0, 1, x, z, NULL));
  CHECK_R1S(r1s_prec_apply(M, R1S_F64, 1, 1, x, zt, NULL));
  CHECK_R1S(r1s_matvec_prec(A, M, R1S_F64, 1, x, yf, zf, NULL));

  /* GMRES(30) solve of J xs = b */
  r1s_gmres_opts opts = {0};
  opts.restart = 30;
  opts.max_cycles = 50;
  opts.rtol = 1e-12;
  opts.op = R1S_OP_STRUCTURED;
  opts.mode = R1S_MODE_F64;
  opts.inner_rtol = 1e-5;
  opts.max_outer = 10;
  CHECK_R1S(r1s_gmres_work_size(A, &opts, 1, &bytes));
  void* work = NULL;
  CHECK_HIP(hipMalloc(&work, bytes));
  r1s_gmres_stats stats;
  CHECK_R1S(r1s_gmres(A, NULL, M, &opts, 1, b, xs, work, bytes, &stats, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  FILE* fo = fopen(argv[2], "wb");
  if (!fo) {
    perror(argv[2]);
    return 1;
  }
  if (save_dev(fo, y, n) || save_dev(fo, yt, n) || save_dev(fo, z, n) || save_dev(fo, zt, n) ||
      save_dev(fo, xs, n) || save_dev(fo, yf, n) || save_dev(fo, zf, n)) {
    fprintf(stderr, "writing results failed\n");
    return 1;
  }
  const int32_t tail[2] = {stats.iters, stats.converged};
  if (fwrite(tail, sizeof tail, 1, fo) != 1) return 1;
  fclose(fo);

  CHECK_R1S(r1s_prec_destroy(M));
  CHECK_R1S(r1s_mat_destroy(A));
  hipFree(work);
  hipFree(prec_mem);
  hipFree(mat_mem);
  return 0;
}
