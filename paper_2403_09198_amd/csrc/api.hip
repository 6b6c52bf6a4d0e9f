// C ABI of libr1s (declared in include/r1s.h): argument validation, layout of
// the caller-provided device buffers, handles and the GMRES driver loop.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <memory>

#include "pattern.hpp"
#include "r1s.h"
#include "r1s_kernels.hpp"

using namespace r1s;

// ------------------------------------------------------------ errors -----
static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                             \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(R1S_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                            \
  } while (0)

extern "C" const char* r1s_last_error(void) { return g_err; }

// ------------------------------------------------------------ helpers ----
static inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }
static inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Carves 256-byte aligned sub-buffers out of one caller buffer.  With a null
// base it only counts bytes, so size queries and init share one layout.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

static int check_dims(int nx, int ny, int L) {
  if (nx < 1 || ny < 1 || L < 1)
    return fail(R1S_ERR_ARG, "nx, ny, L must be >= 1 (got %d, %d, %d)", nx, ny, L);
  if ((long long)nx * ny > (1LL << 30)) return fail(R1S_ERR_ARG, "mesh too large");
  if (L + 3 > R1S_MAX_M)
    return fail(R1S_ERR_UNSUPPORTED, "block size m = L + 3 = %d exceeds %d", L + 3, R1S_MAX_M);
  return R1S_OK;
}

// NULL layout: one pair per block, tridiagonal band, no coupling.
static r1s_layout layout_or_default(const r1s_layout* lay) {
  return lay ? *lay : r1s_layout{1, 1, 1, 0};
}

static int check_layout(const r1s_layout& lay) {
  if (lay.r_diag < 1 || lay.r_off < 0)
    return fail(R1S_ERR_ARG, "need r_diag >= 1 and r_off >= 0 (got %d, %d)", lay.r_diag,
                lay.r_off);
  if (!ranks_supported(lay.r_diag, lay.r_off))
    return fail(R1S_ERR_UNSUPPORTED, "pair counts r_diag = %d, r_off = %d exceed %d, %d",
                lay.r_diag, lay.r_off, RANK_DIAG_MAX, RANK_OFF_MAX);
  if (lay.band < 1 || lay.arrow < 0 || lay.arrow > 2)
    return fail(R1S_ERR_ARG, "need band >= 1 and arrow 0, 1 or 2 (got %d, %d)", lay.band, lay.arrow);
  if (lay.band > R1S_MAX_BAND)
    return fail(R1S_ERR_UNSUPPORTED, "band %d exceeds %d", lay.band, R1S_MAX_BAND);
  return R1S_OK;
}

// nbmax: neighbour slots per cell record (4 on the structured mesh; the
// largest number of off-diagonal blocks of a block row on a general mesh).
static Mesh make_mesh(int nx, int ny, int L, const r1s_layout& lay, bool graph = false,
                      int nbmax = 4) {
  Mesh g{};
  g.nx = nx; g.ny = ny; g.L = L; g.m = L + 3; g.mp = pad_m(L + 3);
  g.N = nx * ny;
  g.n = (long long)g.N * g.m;
  g.rd = lay.r_diag; g.ro = lay.r_off;
  g.graph = graph ? 1 : 0;
  g.nbmax = nbmax;
  g.P = g.rd + nbmax * g.ro;
  g.band = lay.band; g.arrow = lay.arrow;
  g.fb = F_NBR + nbmax;
  g.fa = g.fb + 2 * (g.band - 1);
  g.fu = g.fa + 2 * arrow_slots(g);
  g.F = g.fu + 2 * g.P;
  return g;
}

static long long n_blocks(int nx, int ny) { return 5LL * nx * ny - 2LL * nx - 2LL * ny; }

// ------------------------------------------------------------- matrix ----
struct r1s_mat_s {
  Mesh g;
  int flags;
  double* rec64;
  float* rec32;
  // general mesh: the caller's block structure (host copy) and the device
  // neighbour tables carved from the matrix buffer
  std::vector<int> indptr, indices;
  int *d_nbr, *d_tslot, *d_offb;
  // general pattern of S_cc: the host plan and its device tables
  std::shared_ptr<PatternPlan> plan;
  int* d_pat;
};

// Blocks of the Jacobian: 5N - 2nx - 2ny on the structured mesh, the
// length of block_indices on a general one.
static long long mat_blocks(const r1s_mat_s* A) {
  return A->g.graph ? (long long)A->indices.size() : n_blocks(A->g.nx, A->g.ny);
}

static void mat_layout(Carver& cv, const Mesh& g, int flags, double** r64, float** r32) {
  const size_t cnt = (size_t)g.N * g.F * g.mp;
  *r64 = cv.take<double>(cnt);
  *r32 = (flags & R1S_KEEP_F32) ? cv.take<float>(cnt) : nullptr;
}

extern "C" int r1s_mat_size(int nx, int ny, int L, const r1s_layout* layout, int flags,
                            size_t* bytes) {
  if (int e = check_dims(nx, ny, L)) return e;
  const r1s_layout lay = layout_or_default(layout);
  if (int e = check_layout(lay)) return e;
  if (lay.arrow == 2 && L < 2)
    return fail(R1S_ERR_ARG, "arrow = 2 needs L >= 2 (the atom and a molecule level)");
  if (!bytes) return fail(R1S_ERR_ARG, "bytes is NULL");
  if (flags & ~R1S_KEEP_F32) return fail(R1S_ERR_ARG, "unknown flags 0x%x", flags);
  Carver cv(nullptr);
  double* a;
  float* b;
  mat_layout(cv, make_mesh(nx, ny, L, lay), flags, &a, &b);
  *bytes = cv.off;
  return R1S_OK;
}

// Which inputs a layout reads: the seven base arrays (s_sub / s_sup not for
// L = 1), s_band for band > 1, the coupling arrays with arrow.
static int check_inputs(const r1s_inputs* in, const Mesh& g) {
  if (!in) return fail(R1S_ERR_ARG, "inputs is NULL");
  const void* ps[10] = {in->s_diag, in->s_sub, in->s_sup, in->s_flow, in->s_nbr,
                        in->u,      in->v,     in->s_band, in->s_lev_flow, in->s_flow_lev};
  const char* names[10] = {"s_diag", "s_sub", "s_sup", "s_flow", "s_nbr",
                           "u",      "v",     "s_band", "s_lev_flow", "s_flow_lev"};
  const bool used[10] = {true, g.L > 1, g.L > 1, true, true, true, true,
                         g.band > 1, g.arrow != 0, g.arrow != 0};
  for (int i = 0; i < 10; ++i) {
    if (!used[i]) continue;
    if (!ps[i]) return fail(R1S_ERR_ARG, "input %s is NULL", names[i]);
    if (!aligned(ps[i], 8)) return fail(R1S_ERR_ARG, "input %s is not 8-byte aligned", names[i]);
  }
  return R1S_OK;
}

static int do_pack(r1s_mat A, const r1s_inputs* in, hipStream_t s) {
  PackIn p{in->s_diag, in->s_sub, in->s_sup, in->s_flow, in->s_nbr, in->u, in->v,
           in->s_band, in->s_lev_flow, in->s_flow_lev};
  HIP_TRY(launch_pack(A->g, p, A->rec64, A->rec32, s));
  return R1S_OK;
}

extern "C" int r1s_mat_init(int nx, int ny, int L, const r1s_layout* layout, int flags,
                            const r1s_inputs* in, void* mem, size_t mem_bytes, void* stream,
                            r1s_mat* out) {
  size_t need;
  if (int e = r1s_mat_size(nx, ny, L, layout, flags, &need)) return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  const Mesh g = make_mesh(nx, ny, L, layout_or_default(layout));
  if (int e = check_inputs(in, g)) return e;
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need)
    return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  r1s_mat A = new (std::nothrow) r1s_mat_s();
  if (!A) return fail(R1S_ERR_ALLOC, "host allocation failed");
  A->g = g;
  A->flags = flags;
  Carver cv(mem);
  mat_layout(cv, A->g, flags, &A->rec64, &A->rec32);
  if (int e = do_pack(A, in, as_stream(stream))) {
    delete A;
    return e;
  }
  hipError_t he = hipStreamSynchronize(as_stream(stream));
  if (he != hipSuccess) {
    delete A;
    return fail(R1S_ERR_HIP, "pack: %s", hipGetErrorString(he));
  }
  *out = A;
  return R1S_OK;
}

extern "C" int r1s_mat_update(r1s_mat A, const r1s_inputs* in, void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (A->g.graph) return fail(R1S_ERR_ARG, "general-mesh matrix: use r1s_mat_update_graph");
  if (A->g.pat) return fail(R1S_ERR_ARG, "general-pattern matrix: use r1s_mat_update_pattern");
  if (int e = check_inputs(in, A->g)) return e;
  if (int e = do_pack(A, in, as_stream(stream))) return e;
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  return R1S_OK;
}

extern "C" int r1s_mat_destroy(r1s_mat A) {
  delete A;
  return R1S_OK;
}

// ---------------------------------------------------- general pattern ----
// A structured mesh whose diagonal blocks share a general pattern of S_cc.
static Mesh pattern_mesh(int nx, int ny, int L, const r1s_layout& lay, const PatternPlan& pl) {
  r1s_layout base = lay;
  base.band = 1;
  base.arrow = 0;
  Mesh g = make_mesh(nx, ny, L, base);
  g.pat = 1;
  g.pnnz = pl.nnz;
  g.ne = pl.ne;
  g.net = pl.net;
  g.ns = pl.ns;
  for (int t = 0; t < PAT_SLOTS_MAX; ++t) g.px[t] = pl.px[t];
  g.fb = F_BAND;
  g.fa = g.fb + g.ne;
  g.fu = g.fa + 2 * g.ns;
  g.F = g.fu + 2 * g.P;
  return g;
}

static int pattern_prepare(int nx, int ny, int L, const r1s_layout* layout,
                           const int* pattern_indptr, const int* pattern_indices, int flags,
                           PatternPlan* pl, Mesh* g) {
  if (int e = check_dims(nx, ny, L)) return e;
  const r1s_layout lay = layout_or_default(layout);
  if (int e = check_layout(lay)) return e;
  if (lay.band != 1 || lay.arrow != 0)
    return fail(R1S_ERR_ARG, "a general pattern replaces band and arrow (need 1 and 0, got %d, %d)",
                lay.band, lay.arrow);
  if (flags & ~R1S_KEEP_F32) return fail(R1S_ERR_ARG, "unknown flags 0x%x", flags);
  char msg[256] = "";
  if (int e = build_pattern_plan(L + 3, pattern_indptr, pattern_indices, pl, msg, sizeof msg))
    return fail(e, "%s", msg);
  *g = pattern_mesh(nx, ny, L, lay, *pl);
  return R1S_OK;
}

static void pattern_layout(Carver& cv, const Mesh& g, const PatternPlan& pl, int flags,
                           r1s_mat_s* A) {
  mat_layout(cv, g, flags, &A->rec64, &A->rec32);
  std::vector<int> tab;
  Mesh tmp = g;
  pattern_mat_tables(pl, tab, nullptr, &tmp);
  A->d_pat = cv.take<int>(tab.size());
}

extern "C" int r1s_mat_size_pattern(int nx, int ny, int L, const r1s_layout* layout,
                                    const int* pattern_indptr, const int* pattern_indices,
                                    int flags, size_t* bytes) {
  if (!bytes) return fail(R1S_ERR_ARG, "bytes is NULL");
  PatternPlan pl;
  Mesh g;
  if (int e = pattern_prepare(nx, ny, L, layout, pattern_indptr, pattern_indices, flags, &pl, &g))
    return e;
  Carver cv(nullptr);
  r1s_mat_s tmp;
  pattern_layout(cv, g, pl, flags, &tmp);
  *bytes = cv.off;
  return R1S_OK;
}

static int check_pattern_inputs(const r1s_pattern_inputs* in) {
  if (!in) return fail(R1S_ERR_ARG, "inputs is NULL");
  const void* ps[4] = {in->s_cc, in->s_nbr, in->u, in->v};
  const char* names[4] = {"s_cc", "s_nbr", "u", "v"};
  for (int i = 0; i < 4; ++i) {
    if (!ps[i]) return fail(R1S_ERR_ARG, "input %s is NULL", names[i]);
    if (!aligned(ps[i], 8)) return fail(R1S_ERR_ARG, "input %s is not 8-byte aligned", names[i]);
  }
  return R1S_OK;
}

static int do_pack_pattern(r1s_mat A, const r1s_pattern_inputs* in, hipStream_t s) {
  PackIn p{};
  p.s_nbr = in->s_nbr;
  p.u = in->u;
  p.v = in->v;
  p.s_cc = in->s_cc;
  HIP_TRY(launch_pack(A->g, p, A->rec64, A->rec32, s));
  return R1S_OK;
}

extern "C" int r1s_mat_init_pattern(int nx, int ny, int L, const r1s_layout* layout,
                                    const int* pattern_indptr, const int* pattern_indices,
                                    int flags, const r1s_pattern_inputs* in, void* mem,
                                    size_t mem_bytes, void* stream, r1s_mat* out) {
  size_t need;
  if (int e = r1s_mat_size_pattern(nx, ny, L, layout, pattern_indptr, pattern_indices, flags, &need))
    return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  if (int e = check_pattern_inputs(in)) return e;
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need) return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  auto pl = std::make_shared<PatternPlan>();
  Mesh g;
  pattern_prepare(nx, ny, L, layout, pattern_indptr, pattern_indices, flags, pl.get(), &g);
  r1s_mat A = new (std::nothrow) r1s_mat_s();
  if (!A) return fail(R1S_ERR_ALLOC, "host allocation failed");
  A->flags = flags;
  A->plan = pl;
  Carver cv(mem);
  pattern_layout(cv, g, *pl, flags, A);
  std::vector<int> tab;
  pattern_mat_tables(*pl, tab, A->d_pat, &g);
  A->g = g;
  hipStream_t s = as_stream(stream);
  int rc = R1S_OK;
  do {
    hipError_t e;
    if ((e = hipMemcpyAsync(A->d_pat, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "copy: %s", hipGetErrorString(e)); break; }
    if ((rc = do_pack_pattern(A, in, s))) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "pack: %s", hipGetErrorString(e)); break; }
  } while (0);
  if (rc) {
    (void)hipStreamSynchronize(s);
    delete A;
    return rc;
  }
  *out = A;
  return R1S_OK;
}

extern "C" int r1s_mat_update_pattern(r1s_mat A, const r1s_pattern_inputs* in, void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (!A->g.pat) return fail(R1S_ERR_ARG, "not a general-pattern matrix: use r1s_mat_update");
  if (int e = check_pattern_inputs(in)) return e;
  if (int e = do_pack_pattern(A, in, as_stream(stream))) return e;
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  return R1S_OK;
}

// ------------------------------------------------------- general mesh ----
// Validates the block structure and builds the slot tables: nbr[c][s] = the
// s-th off-diagonal block column of row c (input order, -1 past the row's
// degree), tslot[c][s] = the slot of c in that neighbour's row, offb[c] =
// number of off-diagonal blocks in the rows before c.
struct GraphTables {
  int nbmax = 0;
  long long n_off = 0;
  std::vector<int> nbr, tslot, offb;
};

static int build_graph(int N, const int* indptr, const int* indices, GraphTables* t) {
  if (N < 1) return fail(R1S_ERR_ARG, "n_cells must be >= 1 (got %d)", N);
  if (N > (1 << 30)) return fail(R1S_ERR_ARG, "mesh too large");
  if (!indptr || !indices) return fail(R1S_ERR_ARG, "block_indptr or block_indices is NULL");
  if (indptr[0] != 0) return fail(R1S_ERR_ARG, "block_indptr[0] must be 0");
  int nbmax = 0;
  for (int c = 0; c < N; ++c) {
    const int b0 = indptr[c], b1 = indptr[c + 1];
    if (b1 < b0) return fail(R1S_ERR_ARG, "block_indptr decreases at row %d", c);
    int ndiag = 0;
    for (int b = b0; b < b1; ++b) {
      const int j = indices[b];
      if (j < 0 || j >= N) return fail(R1S_ERR_ARG, "block column %d of row %d out of range", j, c);
      if (j == c) ++ndiag;
      for (int b2 = b0; b2 < b; ++b2)
        if (indices[b2] == j) return fail(R1S_ERR_ARG, "row %d lists block column %d twice", c, j);
    }
    if (ndiag != 1) return fail(R1S_ERR_ARG, "row %d must list its diagonal block once", c);
    nbmax = std::max(nbmax, b1 - b0 - 1);
  }
  if (nbmax > GRAPH_NBR_MAX)
    return fail(R1S_ERR_UNSUPPORTED, "a cell has %d neighbours (at most %d)", nbmax, GRAPH_NBR_MAX);
  t->nbmax = nbmax;
  t->n_off = (long long)indptr[N] - N;
  t->nbr.assign((size_t)N * nbmax, -1);
  t->tslot.assign((size_t)N * nbmax, -1);
  t->offb.resize(N);
  for (int c = 0; c < N; ++c) {
    t->offb[c] = indptr[c] - c;
    int s = 0;
    for (int b = indptr[c]; b < indptr[c + 1]; ++b)
      if (indices[b] != c) t->nbr[(size_t)c * nbmax + s++] = indices[b];
  }
  for (int c = 0; c < N; ++c)
    for (int s = 0; s < nbmax; ++s) {
      const int j = t->nbr[(size_t)c * nbmax + s];
      if (j < 0) break;
      for (int u = 0; u < nbmax; ++u)
        if (t->nbr[(size_t)j * nbmax + u] == c) t->tslot[(size_t)c * nbmax + s] = u;
      if (t->tslot[(size_t)c * nbmax + s] < 0)
        return fail(R1S_ERR_ARG, "block (%d, %d) has no transposed partner (%d, %d)", c, j, j, c);
    }
  return R1S_OK;
}

static void graph_layout(Carver& cv, const Mesh& g, int flags, r1s_mat_s* A) {
  mat_layout(cv, g, flags, &A->rec64, &A->rec32);
  A->d_nbr = cv.take<int>((size_t)g.N * g.nbmax);
  A->d_tslot = cv.take<int>((size_t)g.N * g.nbmax);
  A->d_offb = cv.take<int>(g.N);
}

extern "C" int r1s_mat_size_graph(int n_cells, int L, const r1s_layout* layout,
                                  const int* block_indptr, const int* block_indices, int flags,
                                  size_t* bytes) {
  if (int e = check_dims(n_cells, 1, L)) return e;
  const r1s_layout lay = layout_or_default(layout);
  if (int e = check_layout(lay)) return e;
  if (lay.arrow == 2)
    return fail(R1S_ERR_UNSUPPORTED, "the atom coupling (arrow = 2) is built for the structured mesh only");
  if (!bytes) return fail(R1S_ERR_ARG, "bytes is NULL");
  if (flags & ~R1S_KEEP_F32) return fail(R1S_ERR_ARG, "unknown flags 0x%x", flags);
  GraphTables t;
  if (int e = build_graph(n_cells, block_indptr, block_indices, &t)) return e;
  Carver cv(nullptr);
  r1s_mat_s tmp;
  graph_layout(cv, make_mesh(n_cells, 1, L, lay, true, t.nbmax), flags, &tmp);
  *bytes = cv.off;
  return R1S_OK;
}

static int check_graph_inputs(const r1s_graph_inputs* in, const Mesh& g, long long n_off) {
  if (!in) return fail(R1S_ERR_ARG, "inputs is NULL");
  const void* ps[12] = {in->s_diag, in->s_sub, in->s_sup, in->s_flow, in->s_band, in->s_lev_flow,
                        in->s_flow_lev, in->s_nbr, in->u_diag, in->v_diag, in->u_off, in->v_off};
  const char* names[12] = {"s_diag", "s_sub", "s_sup", "s_flow", "s_band", "s_lev_flow",
                           "s_flow_lev", "s_nbr", "u_diag", "v_diag", "u_off", "v_off"};
  const bool used[12] = {true, g.L > 1, g.L > 1, true, g.band > 1, g.arrow != 0, g.arrow != 0,
                         n_off > 0, true, true, n_off > 0 && g.ro > 0, n_off > 0 && g.ro > 0};
  for (int i = 0; i < 12; ++i) {
    if (!used[i]) continue;
    if (!ps[i]) return fail(R1S_ERR_ARG, "input %s is NULL", names[i]);
    if (!aligned(ps[i], 8)) return fail(R1S_ERR_ARG, "input %s is not 8-byte aligned", names[i]);
  }
  return R1S_OK;
}

static int do_pack_graph(r1s_mat A, const r1s_graph_inputs* in, hipStream_t s) {
  GraphPackIn p{in->s_diag, in->s_sub,  in->s_sup,  in->s_flow,  in->s_band, in->s_lev_flow,
                in->s_flow_lev, in->s_nbr, in->u_diag, in->v_diag, in->u_off, in->v_off};
  HIP_TRY(launch_pack_graph(A->g, p, A->rec64, A->rec32, s));
  return R1S_OK;
}

extern "C" int r1s_mat_init_graph(int n_cells, int L, const r1s_layout* layout,
                                  const int* block_indptr, const int* block_indices, int flags,
                                  const r1s_graph_inputs* in, void* mem, size_t mem_bytes,
                                  void* stream, r1s_mat* out) {
  size_t need;
  if (int e = r1s_mat_size_graph(n_cells, L, layout, block_indptr, block_indices, flags, &need))
    return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  GraphTables t;
  build_graph(n_cells, block_indptr, block_indices, &t);  // validated by the size call
  Mesh g = make_mesh(n_cells, 1, L, layout_or_default(layout), true, t.nbmax);
  if (int e = check_graph_inputs(in, g, t.n_off)) return e;
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need)
    return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  r1s_mat A = new (std::nothrow) r1s_mat_s();
  if (!A) return fail(R1S_ERR_ALLOC, "host allocation failed");
  A->flags = flags;
  A->indptr.assign(block_indptr, block_indptr + n_cells + 1);
  A->indices.assign(block_indices, block_indices + block_indptr[n_cells]);
  Carver cv(mem);
  graph_layout(cv, g, flags, A);
  g.nbr = A->d_nbr;
  g.tslot = A->d_tslot;
  g.offb = A->d_offb;
  A->g = g;
  hipStream_t s = as_stream(stream);
  int rc = R1S_OK;
  do {
    hipError_t e;
    const size_t tb = t.nbr.size() * sizeof(int);
    if (tb && (e = hipMemcpyAsync(A->d_nbr, t.nbr.data(), tb, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "copy: %s", hipGetErrorString(e)); break; }
    if (tb && (e = hipMemcpyAsync(A->d_tslot, t.tslot.data(), tb, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "copy: %s", hipGetErrorString(e)); break; }
    if ((e = hipMemcpyAsync(A->d_offb, t.offb.data(), t.offb.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "copy: %s", hipGetErrorString(e)); break; }
    if ((rc = do_pack_graph(A, in, s))) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "pack: %s", hipGetErrorString(e)); break; }
  } while (0);
  if (rc) {
    // the copies read the host tables: wait for them before they go away
    (void)hipStreamSynchronize(s);
    delete A;
    return rc;
  }
  *out = A;
  return R1S_OK;
}

extern "C" int r1s_mat_update_graph(r1s_mat A, const r1s_graph_inputs* in, void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (!A->g.graph) return fail(R1S_ERR_ARG, "structured-mesh matrix: use r1s_mat_update");
  if (int e = check_graph_inputs(in, A->g, mat_blocks(A) - A->g.N)) return e;
  if (int e = do_pack_graph(A, in, as_stream(stream))) return e;
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  return R1S_OK;
}

extern "C" int r1s_mat_storage(r1s_mat A, r1s_storage* out) {
  if (!A || !out) return fail(R1S_ERR_ARG, "NULL argument");
  const Mesh& g = A->g;
  const long long B = mat_blocks(A), N = g.N, m = g.m;
  out->n_cells = N;
  out->n_blocks = B;
  out->m = m;
  const long long pairs = N * g.rd + (B - N) * g.ro;
  const long long L = g.L;
  long long diag_block = 3 * m - 2;  // diagonal, tridiagonal band, 3 x 3 corner
  for (int j = 2; j <= g.band; ++j) diag_block += 2 * std::max(L - j, 0LL);
  if (g.arrow) diag_block += 6 * L;
  // the atom's column and row, less the positions the band already holds
  if (g.arrow == 2) diag_block += 2 * std::max(L - 1 - g.band, 0LL);
  if (g.pat) diag_block = g.pnnz;  // a general pattern: its entries
  out->structured_values = N * diag_block + (B - N) * m + 2 * pairs * m;
  out->structured_padded = N * (long long)g.F * g.mp;
  out->bsr_values = B * m * m;
  // structured mesh: neighbours implicit; general mesh: the int32 slot
  // tables (neighbour, reverse slot) and first off-block per cell
  out->index_bytes = g.graph ? 4 * (2 * N * g.nbmax + N) : 0;
  out->matvec_bytes = 8 * out->structured_values + 8 * 2 * N * m + out->index_bytes;
  // A0 factors (as many values as S_cc; with the wide pattern the band LU
  // factors, the coupling factors and the 3 x 3 Schur inverse), W and V,
  // C^{-1}; r read, z written
  const long long a0 = g.pat ? (long long)A->plan->nnzF
                             : wide_pattern(g) ? (2 * g.band + 1 + (g.arrow ? 6 : 0)) * L + 9
                                               : 3 * m - 2;
  const long long pw = smw_pairs(g);  // with the atom: two more Woodbury terms
  out->smw_apply_bytes = 8 * N * (a0 + 2 * pw * m + pw * pw) + 8 * 2 * N * m;
  return R1S_OK;
}

static int check_vec(const void* p, const char* name) {
  if (!p) return fail(R1S_ERR_ARG, "%s is NULL", name);
  if (!aligned(p, 8)) return fail(R1S_ERR_ARG, "%s is not 8-byte aligned", name);
  return R1S_OK;
}

extern "C" int r1s_matvec(r1s_mat A, int precision, int trans, int nrhs, const double* x,
                          double* y, void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (precision != R1S_F64 && precision != R1S_F32)
    return fail(R1S_ERR_ARG, "unknown precision %d", precision);
  if (precision == R1S_F32 && !A->rec32)
    return fail(R1S_ERR_ARG, "float32 matvec needs a matrix made with R1S_KEEP_F32");
  if (int e = check_vec(x, "x")) return e;
  if (int e = check_vec(y, "y")) return e;
  if (x == y) return fail(R1S_ERR_ARG, "x and y must not alias");
  const bool f32 = precision == R1S_F32;
  HIP_TRY(launch_matvec(A->g, f32 ? (const void*)A->rec32 : (const void*)A->rec64, f32, trans != 0,
                        x, y, nrhs, as_stream(stream)));
  return R1S_OK;
}

extern "C" int r1s_residual(r1s_mat A, int nrhs, const double* b, const double* x, double* r,
                            void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (int e = check_vec(b, "b")) return e;
  if (int e = check_vec(x, "x")) return e;
  if (int e = check_vec(r, "r")) return e;
  if (x == r) return fail(R1S_ERR_ARG, "x and r must not alias");
  HIP_TRY(launch_residual(A->g, A->rec64, false, b, x, r, nrhs, as_stream(stream)));
  return R1S_OK;
}

// -------------------------------------------------------- preconditioner --
enum { PREC_SMW = 0, PREC_BSR_LU = 1 };

struct r1s_prec_s {
  int kind;
  int flags;
  Mesh g;
  // SMW, tridiagonal level band with or without level/flow coupling (one
  // wave per cell)
  double *facF, *facT, *invC;
  float *facF32, *facT32, *invC32;
  int* status;
  // SMW, level band wider than tridiagonal (tile-interleaved, 32 cells per tile):
  // band / coupling factors, Schur inverse, W and V rows per direction, C^{-1}
  double *bf, *s3i, *wv, *wvT, *cinv;
  float *bf32, *s3i32, *wv32, *wvT32, *cinv32;
  long long n_bf, n_s3i, n_wv, n_cinv;  // element counts
  // general pattern: the LU position tables (device, in this buffer); the
  // band fields above hold its factors (s3i unused)
  PatLU plu;
  int* d_lu;
  long long n_lu;
  // BSR dense LU
  double* lu;
  int* piv;
};

static void prec_layout(Carver& cv, const r1s_mat_s* A, int flags, r1s_prec_s* P) {
  const Mesh& g = A->g;
  const bool f32 = flags & R1S_KEEP_F32, tr = flags & R1S_WITH_TRANS;
  if (band_walk(g)) {
    if (g.pat) {
      pattern_prec_counts(g, A->plan->nnzF, &P->n_bf, &P->n_wv, &P->n_cinv);
      P->n_s3i = 0;
      std::vector<int> tab;
      pattern_lu_tables(*A->plan, tab, nullptr, &P->plu);
      P->n_lu = (long long)tab.size();
      P->d_lu = cv.take<int>(tab.size());
    } else {
      band_prec_counts(g, &P->n_bf, &P->n_s3i, &P->n_wv, &P->n_cinv);
    }
    P->bf = cv.take<double>(P->n_bf);
    P->s3i = cv.take<double>(P->n_s3i);
    P->wv = cv.take<double>(P->n_wv);
    P->wvT = tr ? cv.take<double>(P->n_wv) : nullptr;
    P->cinv = cv.take<double>(P->n_cinv);
    P->status = cv.take<int>(64);
    P->bf32 = f32 ? cv.take<float>(P->n_bf) : nullptr;
    P->s3i32 = f32 ? cv.take<float>(P->n_s3i) : nullptr;
    P->wv32 = f32 ? cv.take<float>(P->n_wv) : nullptr;
    P->wvT32 = (f32 && tr) ? cv.take<float>(P->n_wv) : nullptr;
    P->cinv32 = f32 ? cv.take<float>(P->n_cinv) : nullptr;
    return;
  }
  const size_t f = (size_t)g.N * smw_rows(g) * g.mp;
  const size_t ic = (size_t)g.N * smw_pairs(g) * smw_pairs(g);
  P->facF = cv.take<double>(f);
  P->facT = (flags & R1S_WITH_TRANS) ? cv.take<double>(f) : nullptr;
  P->invC = cv.take<double>(ic);
  P->status = cv.take<int>(64);
  P->facF32 = (flags & R1S_KEEP_F32) ? cv.take<float>(f) : nullptr;
  P->facT32 = ((flags & R1S_KEEP_F32) && (flags & R1S_WITH_TRANS)) ? cv.take<float>(f) : nullptr;
  P->invC32 = (flags & R1S_KEEP_F32) ? cv.take<float>(ic) : nullptr;
}

static bool smw_has_trans(const r1s_prec_s* M) { return M->facT || M->wvT; }
static bool smw_has_f32(const r1s_prec_s* M) { return M->facF32 || M->bf32; }

extern "C" int r1s_prec_size(r1s_mat A, int flags, size_t* bytes) {
  if (!A || !bytes) return fail(R1S_ERR_ARG, "NULL argument");
  if (flags & ~(R1S_KEEP_F32 | R1S_WITH_TRANS)) return fail(R1S_ERR_ARG, "unknown flags 0x%x", flags);
  Carver cv(nullptr);
  r1s_prec_s tmp = {};
  prec_layout(cv, A, flags, &tmp);
  *bytes = cv.off;
  return R1S_OK;
}

static int read_status(int* dstatus, hipStream_t s, int* host) {
  HIP_TRY(hipMemcpyAsync(host, dstatus, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return R1S_OK;
}

extern "C" int r1s_prec_setup(r1s_mat A, int flags, void* mem, size_t mem_bytes, void* stream,
                              r1s_prec* out) {
  size_t need;
  if (int e = r1s_prec_size(A, flags, &need)) return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need) return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  r1s_prec P = (r1s_prec)calloc(1, sizeof(r1s_prec_s));
  if (!P) return fail(R1S_ERR_ALLOC, "host allocation failed");
  P->kind = PREC_SMW;
  P->flags = flags;
  P->g = A->g;
  Carver cv(mem);
  prec_layout(cv, A, flags, P);
  hipStream_t s = as_stream(stream);
  int st = 0x7fffffff;
  int rc = R1S_OK;
  std::vector<int> lu_tab;  // host copy of a general pattern's LU tables, read by an async copy
  do {
    hipError_t e;
    if ((e = launch_fill_int(P->status, 0x7fffffff, 1, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "fill: %s", hipGetErrorString(e)); break; }
    if (band_walk(A->g)) {
      if (A->g.pat) {
        // the LU tables next to the factors (a copy from pageable memory has
        // taken the data when it returns)
        pattern_lu_tables(*A->plan, lu_tab, P->d_lu, &P->plu);
        if ((e = hipMemcpyAsync(P->d_lu, lu_tab.data(), lu_tab.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "copy: %s", hipGetErrorString(e)); break; }
        if ((e = launch_pattern_setup(A->g, P->plu, A->rec64, P->bf, P->wv, P->wvT, P->cinv, P->status, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "pattern setup: %s", hipGetErrorString(e)); break; }
      } else if ((e = launch_band_setup(A->g, A->rec64, P->bf, P->s3i, P->wv, P->wvT, P->cinv, P->status, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "band setup: %s", hipGetErrorString(e)); break; }
      if (P->bf32) {
        const double* src[5] = {P->bf, P->s3i, P->wv, P->wvT, P->cinv};
        float* dst[5] = {P->bf32, P->s3i32, P->wv32, P->wvT32, P->cinv32};
        const long long cnt[5] = {P->n_bf, P->n_s3i, P->n_wv, P->n_wv, P->n_cinv};
        for (int i = 0; i < 5 && e == hipSuccess; ++i)
          if (dst[i] && cnt[i] > 0) e = launch_cast_f32(src[i], dst[i], cnt[i], s);
        if (e != hipSuccess) { rc = fail(R1S_ERR_HIP, "cast: %s", hipGetErrorString(e)); break; }
      }
    } else if ((e = launch_smw_setup(A->g, A->rec64, P->facF, P->facT, P->invC, P->status, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "smw setup: %s", hipGetErrorString(e)); break; }
    if (!band_walk(A->g) && P->facF32) {
      const long long f = (long long)A->g.N * smw_rows(A->g) * A->g.mp;
      if ((e = launch_cast_f32(P->facF, P->facF32, f, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "cast: %s", hipGetErrorString(e)); break; }
      if (P->facT32 && (e = launch_cast_f32(P->facT, P->facT32, f, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "cast: %s", hipGetErrorString(e)); break; }
      if ((e = launch_cast_f32(P->invC, P->invC32, (long long)A->g.N * smw_pairs(A->g) * smw_pairs(A->g), s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "cast: %s", hipGetErrorString(e)); break; }
    }
    if ((rc = read_status(P->status, s, &st))) break;
    if (st != 0x7fffffff) {
      rc = fail(R1S_ERR_SINGULAR, "SMW setup: singular diagonal block (zero pivot or capacitance) at cell %d", st);
      break;
    }
  } while (0);
  if (rc) {
    free(P);
    return rc;
  }
  *out = P;
  return R1S_OK;
}

extern "C" int r1s_prec_apply(r1s_prec M, int precision, int trans, int nrhs, const double* r,
                              double* z, void* stream) {
  if (!M) return fail(R1S_ERR_ARG, "preconditioner handle is NULL");
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (int e = check_vec(r, "r")) return e;
  if (int e = check_vec(z, "z")) return e;
  if (r == z) return fail(R1S_ERR_ARG, "r and z must not alias");
  if (precision != R1S_F64 && precision != R1S_F32)
    return fail(R1S_ERR_ARG, "unknown precision %d", precision);
  hipStream_t s = as_stream(stream);
  if (M->kind == PREC_BSR_LU) {
    if (trans || precision != R1S_F64)
      return fail(R1S_ERR_UNSUPPORTED, "the dense-LU preconditioner applies M r in float64 only");
    HIP_TRY(launch_bsr_lu_apply(M->g, M->lu, M->piv, r, z, nrhs, s));
    return R1S_OK;
  }
  if (band_walk(M->g)) {
    if (trans && !M->wvT) return fail(R1S_ERR_ARG, "transposed apply needs R1S_WITH_TRANS at setup");
    const bool f32 = precision == R1S_F32;
    if (f32 && !M->bf32) return fail(R1S_ERR_ARG, "float32 apply needs R1S_KEEP_F32 at setup");
    const void* w = f32 ? (trans ? (const void*)M->wvT32 : (const void*)M->wv32)
                        : (trans ? (const void*)M->wvT : (const void*)M->wv);
    if (M->g.pat) {
      HIP_TRY(launch_pattern_apply(M->g, M->plu, f32 ? (const void*)M->bf32 : (const void*)M->bf, w,
                                   f32 ? (const void*)M->cinv32 : (const void*)M->cinv, f32,
                                   trans != 0, r, z, nrhs, s));
      return R1S_OK;
    }
    HIP_TRY(launch_band_apply(M->g, f32 ? (const void*)M->bf32 : (const void*)M->bf,
                              f32 ? (const void*)M->s3i32 : (const void*)M->s3i, w,
                              f32 ? (const void*)M->cinv32 : (const void*)M->cinv, f32, trans != 0,
                              r, z, nrhs, s));
    return R1S_OK;
  }
  if (trans && !M->facT) return fail(R1S_ERR_ARG, "transposed apply needs R1S_WITH_TRANS at setup");
  if (precision == R1S_F32) {
    if (!M->facF32) return fail(R1S_ERR_ARG, "float32 apply needs R1S_KEEP_F32 at setup");
    HIP_TRY(launch_smw_apply(M->g, trans ? (const void*)M->facT32 : (const void*)M->facF32, M->invC32,
                             true, trans != 0, r, z, nrhs, s));
  } else {
    HIP_TRY(launch_smw_apply(M->g, trans ? (const void*)M->facT : (const void*)M->facF, M->invC,
                             false, trans != 0, r, z, nrhs, s));
  }
  return R1S_OK;
}

static bool same_layout(const Mesh& a, const Mesh& b) {
  return a.nx == b.nx && a.ny == b.ny && a.N == b.N && a.L == b.L && a.m == b.m && a.rd == b.rd &&
         a.ro == b.ro && a.band == b.band && a.arrow == b.arrow && a.graph == b.graph &&
         a.pat == b.pat && a.pnnz == b.pnnz;
}

extern "C" int r1s_matvec_prec(r1s_mat A, r1s_prec M, int precision, int nrhs, const double* x,
                               double* y, double* z, void* stream) {
  if (!A) return fail(R1S_ERR_ARG, "matrix handle is NULL");
  if (!M) return fail(R1S_ERR_ARG, "preconditioner handle is NULL");
  if (M->kind != PREC_SMW)
    return fail(R1S_ERR_UNSUPPORTED, "r1s_matvec_prec takes an SMW preconditioner");
  if (!same_layout(A->g, M->g)) return fail(R1S_ERR_ARG, "A and M have different layouts");
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (precision != R1S_F64 && precision != R1S_F32)
    return fail(R1S_ERR_ARG, "unknown precision %d", precision);
  const bool f32 = precision == R1S_F32;
  if (f32 && !A->rec32)
    return fail(R1S_ERR_ARG, "float32 matvec needs a matrix made with R1S_KEEP_F32");
  if (f32 && !smw_has_f32(M)) return fail(R1S_ERR_ARG, "float32 apply needs R1S_KEEP_F32 at setup");
  if (int e = check_vec(x, "x")) return e;
  if (int e = check_vec(y, "y")) return e;
  if (int e = check_vec(z, "z")) return e;
  if (x == y || x == z || y == z) return fail(R1S_ERR_ARG, "x, y and z must not alias");
  if (nrhs == 1 && matvec_prec_fused(A->g, f32)) {
    HIP_TRY(launch_matvec_prec(A->g, f32 ? (const void*)A->rec32 : (const void*)A->rec64,
                               f32 ? (const void*)M->facF32 : (const void*)M->facF,
                               f32 ? (const void*)M->invC32 : (const void*)M->invC, f32, x, y, z,
                               as_stream(stream)));
    return R1S_OK;
  }
  if (int e = r1s_matvec(A, precision, 0, nrhs, x, y, stream)) return e;
  return r1s_prec_apply(M, precision, 0, nrhs, y, z, stream);
}

extern "C" int r1s_prec_destroy(r1s_prec M) {
  free(M);
  return R1S_OK;
}

// ------------------------------------------------------------------ BSR ---
struct r1s_bsr_s {
  Mesh g;
  long long nblocks;
  int *indptr, *indices, *blk_row, *blk_dir, *diag_block;
  double* data;
};

static void bsr_layout(Carver& cv, const Mesh& g, long long nblocks, r1s_bsr_s* B) {
  B->nblocks = nblocks;
  B->data = cv.take<double>((size_t)B->nblocks * g.m * g.m);
  B->indptr = cv.take<int>(g.N + 1);
  B->indices = cv.take<int>(B->nblocks);
  B->blk_row = cv.take<int>(B->nblocks);
  B->blk_dir = cv.take<int>(B->nblocks);
  B->diag_block = cv.take<int>(g.N);
}

extern "C" int r1s_bsr_size(r1s_mat A, size_t* bytes) {
  if (!A || !bytes) return fail(R1S_ERR_ARG, "NULL argument");
  Carver cv(nullptr);
  r1s_bsr_s tmp;
  bsr_layout(cv, A->g, mat_blocks(A), &tmp);
  *bytes = cv.off;
  return R1S_OK;
}

extern "C" int r1s_bsr_init(r1s_mat A, void* mem, size_t mem_bytes, void* stream, r1s_bsr* out) {
  size_t need;
  if (int e = r1s_bsr_size(A, &need)) return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need) return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  const Mesh& g = A->g;
  if (mat_blocks(A) * g.m * g.m > (1LL << 62)) return fail(R1S_ERR_UNSUPPORTED, "BSR too large");
  r1s_bsr B = (r1s_bsr)calloc(1, sizeof(r1s_bsr_s));
  if (!B) return fail(R1S_ERR_ALLOC, "host allocation failed");
  B->g = g;
  Carver cv(mem);
  bsr_layout(cv, g, mat_blocks(A), B);
  // block structure in BSR order: block rows by cell; structured mesh:
  // columns ascending (S, W, C, E, N); general mesh: the caller's order
  std::vector<int> indptr(g.N + 1), indices, row, dir, diag(g.N);
  indices.reserve(B->nblocks);
  for (int c = 0; c < g.N; ++c) {
    indptr[c] = (int)indices.size();
    if (g.graph) {
      int slot = 0;
      for (int b = A->indptr[c]; b < A->indptr[c + 1]; ++b) {
        const int j = A->indices[b];
        if (j == c) diag[c] = (int)indices.size();
        indices.push_back(j);
        row.push_back(c);
        dir.push_back(j == c ? D_C : GSLOT + slot++);
      }
      continue;
    }
    const int iy = c / g.nx, ix = c % g.nx;
    const int nbs[5] = {iy > 0 ? c - g.nx : -1, ix > 0 ? c - 1 : -1, c,
                        ix < g.nx - 1 ? c + 1 : -1, iy < g.ny - 1 ? c + g.nx : -1};
    for (int d = 0; d < 5; ++d) {
      if (nbs[d] < 0) continue;
      if (d == D_C) diag[c] = (int)indices.size();
      indices.push_back(nbs[d]);
      row.push_back(c);
      dir.push_back(d);
    }
  }
  indptr[g.N] = (int)indices.size();
  hipStream_t s = as_stream(stream);
  int rc = R1S_OK;
  do {
    hipError_t e;
#define TRY_(x) if ((e = (x)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "%s: %s", #x, hipGetErrorString(e)); break; }
    TRY_(hipMemcpyAsync(B->indptr, indptr.data(), indptr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    TRY_(hipMemcpyAsync(B->indices, indices.data(), indices.size() * sizeof(int), hipMemcpyHostToDevice, s));
    TRY_(hipMemcpyAsync(B->blk_row, row.data(), row.size() * sizeof(int), hipMemcpyHostToDevice, s));
    TRY_(hipMemcpyAsync(B->blk_dir, dir.data(), dir.size() * sizeof(int), hipMemcpyHostToDevice, s));
    TRY_(hipMemcpyAsync(B->diag_block, diag.data(), diag.size() * sizeof(int), hipMemcpyHostToDevice, s));
    TRY_(launch_bsr_assemble(g, A->rec64, B->blk_row, B->blk_dir, B->nblocks, B->data, s));
    TRY_(hipStreamSynchronize(s));
#undef TRY_
  } while (0);
  if (rc) {
    free(B);
    return rc;
  }
  *out = B;
  return R1S_OK;
}

extern "C" int r1s_bsr_matvec(r1s_bsr B, int nrhs, const double* x, double* y, void* stream) {
  if (!B) return fail(R1S_ERR_ARG, "BSR handle is NULL");
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (int e = check_vec(x, "x")) return e;
  if (int e = check_vec(y, "y")) return e;
  if (x == y) return fail(R1S_ERR_ARG, "x and y must not alias");
  HIP_TRY(launch_bsr_matvec(B->g, B->indptr, B->indices, B->data, x, y, nrhs, as_stream(stream)));
  return R1S_OK;
}

static void bsr_prec_layout(Carver& cv, const Mesh& g, r1s_prec_s* P, int** info) {
  P->lu = cv.take<double>((size_t)g.N * g.m * g.m);
  P->piv = cv.take<int>((size_t)g.N * g.m);
  P->status = cv.take<int>(64);
  *info = cv.take<int>(g.N);
}

// Dense LU of blocks too large for LDS: rocSOLVER's batched getrf (baseline
// setup only; it allocates its own workspace through rocBLAS).
static int library_lu(const r1s_bsr_s* B, r1s_prec_s* P, int* info, hipStream_t s) {
  HIP_TRY(launch_bsr_gather_diag(B->g, B->diag_block, B->data, P->lu, s));
  rocblas_handle h;
  if (rocblas_create_handle(&h) != rocblas_status_success)
    return fail(R1S_ERR_HIP, "rocblas_create_handle failed");
  rocblas_set_stream(h, s);
  const int m = B->g.m;
  const rocblas_status st = rocsolver_dgetrf_strided_batched(
      h, m, m, P->lu, m, (rocblas_stride)m * m, P->piv, (rocblas_stride)m, info, B->g.N);
  rocblas_destroy_handle(h);
  if (st != rocblas_status_success)
    return fail(R1S_ERR_HIP, "rocsolver_dgetrf_strided_batched failed (%d)", (int)st);
  HIP_TRY(launch_bsr_piv_convert(B->g, P->piv, info, P->status, s));
  return R1S_OK;
}

extern "C" int r1s_bsr_prec_size(r1s_bsr B, size_t* bytes) {
  if (!B || !bytes) return fail(R1S_ERR_ARG, "NULL argument");
  Carver cv(nullptr);
  r1s_prec_s tmp;
  int* info;
  bsr_prec_layout(cv, B->g, &tmp, &info);
  *bytes = cv.off;
  return R1S_OK;
}

extern "C" int r1s_bsr_prec_setup(r1s_bsr B, void* mem, size_t mem_bytes, void* stream,
                                  r1s_prec* out) {
  size_t need;
  if (int e = r1s_bsr_prec_size(B, &need)) return e;
  if (!out) return fail(R1S_ERR_ARG, "out is NULL");
  if (!mem || !aligned(mem, 256)) return fail(R1S_ERR_ARG, "mem is NULL or not 256-byte aligned");
  if (mem_bytes < need) return fail(R1S_ERR_ARG, "mem_bytes %zu < required %zu", mem_bytes, need);
  r1s_prec P = (r1s_prec)calloc(1, sizeof(r1s_prec_s));
  if (!P) return fail(R1S_ERR_ALLOC, "host allocation failed");
  P->kind = PREC_BSR_LU;
  P->g = B->g;
  Carver cv(mem);
  int* info;
  bsr_prec_layout(cv, B->g, P, &info);
  hipStream_t s = as_stream(stream);
  int st = 0x7fffffff, rc = R1S_OK;
  do {
    hipError_t e;
    if ((e = launch_fill_int(P->status, 0x7fffffff, 1, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "fill: %s", hipGetErrorString(e)); break; }
    if (bsr_lu_fits_lds(B->g)) {
      if ((e = launch_bsr_lu_setup(B->g, B->diag_block, B->data, P->lu, P->piv, P->status, s)) != hipSuccess) { rc = fail(R1S_ERR_HIP, "bsr lu: %s", hipGetErrorString(e)); break; }
    } else if ((rc = library_lu(B, P, info, s))) {
      break;
    }
    if ((rc = read_status(P->status, s, &st))) break;
    if (st != 0x7fffffff) { rc = fail(R1S_ERR_SINGULAR, "dense LU: zero pivot in the diagonal block of cell %d", st); break; }
  } while (0);
  if (rc) {
    free(P);
    return rc;
  }
  *out = P;
  return R1S_OK;
}

extern "C" int r1s_bsr_destroy(r1s_bsr B) {
  free(B);
  return R1S_OK;
}

// ---------------------------------------------------------------- GMRES ---
struct GmresWork {
  double *V, *w, *z, *t, *part, *hdev, *ydev, *scal, *r64, *d;
  int* need;  // per right-hand side: the second Gram-Schmidt pass ran
  double* dstate;       // delayed reorthogonalisation: per-rhs H, s, a, g, r, rho
  long long dstride;
  int nblk;
};

static void gmres_layout(Carver& cv, const Mesh& g, int k, int nrhs, bool mixed, GmresWork* W) {
  const size_t n = (size_t)g.n;
  W->nblk = dot_blocks(g.n);
  W->V = cv.take<double>((size_t)nrhs * (k + 1) * n);
  W->w = cv.take<double>((size_t)nrhs * n);
  W->z = cv.take<double>((size_t)nrhs * n);
  W->t = cv.take<double>((size_t)nrhs * n);
  W->part = cv.take<double>((size_t)nrhs * (2 * k + 3) * W->nblk);
  W->hdev = cv.take<double>((size_t)nrhs * (k + 2) * 2);
  W->ydev = cv.take<double>((size_t)nrhs * (k + 1));
  W->scal = cv.take<double>((size_t)nrhs * 4);
  W->r64 = mixed ? cv.take<double>((size_t)nrhs * n) : nullptr;
  W->d = mixed ? cv.take<double>((size_t)nrhs * n) : nullptr;
  W->need = cv.take<int>((size_t)nrhs);
  W->dstride = (long long)k * (k + 1) + 3LL * k + 2 + 4;
  W->dstate = cv.take<double>((size_t)nrhs * W->dstride);
}

// Pinned host staging for the Arnoldi coefficients, written by the last
// kernel of each step, so that the host reads them behind the next step's
// kernels.  Two slots (alternating steps), each h1, h2 [nrhs][k + 2] and
// need [nrhs] (as doubles), plus one event per slot.  Pooled per device and reused across solves; the pool is
// never freed (the memory returns to the system at process exit).
struct Staging {
  int device = -1;
  size_t bytes = 0;
  char* mem = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};
static std::mutex g_staging_mu;
static std::vector<Staging*> g_staging_free;

static int staging_acquire(size_t bytes, Staging** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Staging* st = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_staging_mu);
    for (size_t i = 0; i < g_staging_free.size(); ++i)
      if (g_staging_free[i]->device == dev) {
        st = g_staging_free[i];
        g_staging_free.erase(g_staging_free.begin() + i);
        break;
      }
  }
  if (!st) {
    st = new (std::nothrow) Staging();
    if (!st) return fail(R1S_ERR_ALLOC, "host allocation failed");
    st->device = dev;
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&st->ev[i], hipEventDisableTiming) != hipSuccess) {
        delete st;
        return fail(R1S_ERR_HIP, "event creation failed");
      }
  }
  if (st->bytes < bytes) {
    if (st->mem) (void)hipHostFree(st->mem);
    st->mem = nullptr;
    st->bytes = 0;
    if (hipHostMalloc((void**)&st->mem, bytes, hipHostMallocDefault) != hipSuccess) {
      std::lock_guard<std::mutex> lk(g_staging_mu);
      g_staging_free.push_back(st);
      return fail(R1S_ERR_ALLOC, "pinned host allocation of %zu bytes failed", bytes);
    }
    st->bytes = bytes;
  }
  *out = st;
  return R1S_OK;
}

// Returns the staging buffer to the pool once the solve's stream has drained
// (on an early error return kernels may still write into it).
struct StagingLease {
  Staging* st = nullptr;
  hipStream_t stream = nullptr;
  bool drained = false;  // the host has seen the stream's last kernel raise its flag
  ~StagingLease() {
    if (st) {
      if (!drained) (void)hipStreamSynchronize(stream);
      std::lock_guard<std::mutex> lk(g_staging_mu);
      g_staging_free.push_back(st);
    }
  }
};

static int check_opts(const r1s_gmres_opts* o) {
  if (!o) return fail(R1S_ERR_ARG, "opts is NULL");
  if (o->restart < 1 || o->restart > 1000) return fail(R1S_ERR_ARG, "restart must be in [1, 1000]");
  if (o->max_cycles < 1) return fail(R1S_ERR_ARG, "max_cycles must be >= 1");
  if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) return fail(R1S_ERR_ARG, "rtol must be in (0, 1)");
  if (o->op != R1S_OP_STRUCTURED && o->op != R1S_OP_BSR) return fail(R1S_ERR_ARG, "unknown op");
  if (o->mode != R1S_MODE_F64 && o->mode != R1S_MODE_MIXED_IR) return fail(R1S_ERR_ARG, "unknown mode");
  if (o->ortho != R1S_ORTHO_SELECTIVE && o->ortho != R1S_ORTHO_CGS2 && o->ortho != R1S_ORTHO_DELAYED)
    return fail(R1S_ERR_ARG, "unknown orthogonalisation %d", o->ortho);
  if (o->mode == R1S_MODE_MIXED_IR) {
    if (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0)) return fail(R1S_ERR_ARG, "inner_rtol must be in (0, 1)");
    if (o->max_outer < 1) return fail(R1S_ERR_ARG, "max_outer must be >= 1");
    if (o->op != R1S_OP_STRUCTURED) return fail(R1S_ERR_ARG, "mixed mode needs the structured operator");
  }
  return R1S_OK;
}

extern "C" int r1s_gmres_work_size(r1s_mat A, const r1s_gmres_opts* opts, int nrhs, size_t* bytes) {
  if (!A || !bytes) return fail(R1S_ERR_ARG, "NULL argument");
  if (int e = check_opts(opts)) return e;
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  Carver cv(nullptr);
  GmresWork W;
  gmres_layout(cv, A->g, opts->restart, nrhs, opts->mode == R1S_MODE_MIXED_IR, &W);
  *bytes = cv.off;
  return R1S_OK;
}

// The operator pair one GMRES solve works with.
struct OpCtx {
  r1s_mat A;
  r1s_bsr B;
  r1s_prec M;
  bool f32;   // float32 operator + preconditioner (inner solves)
  bool trans;
  bool bsr;
  hipStream_t s;
};

static int op_apply(const OpCtx& c, const double* in, double* out, int nrhs) {
  if (c.bsr) {
    HIP_TRY(launch_bsr_matvec(c.B->g, c.B->indptr, c.B->indices, c.B->data, in, out, nrhs, c.s));
  } else {
    HIP_TRY(launch_matvec(c.A->g, c.f32 ? (const void*)c.A->rec32 : (const void*)c.A->rec64, c.f32,
                          c.trans, in, out, nrhs, c.s));
  }
  return R1S_OK;
}

static int prec_apply(const OpCtx& c, const double* in, double* out, int nrhs) {
  if (int e = r1s_prec_apply(c.M, c.f32 ? R1S_F32 : R1S_F64, c.trans ? 1 : 0, nrhs, in, out, c.s))
    return e;
  return R1S_OK;
}

// out = b - op(x), float64 for the structured operator in f64 mode, else via op
static int op_residual(const OpCtx& c, const double* b, const double* x, double* out, int nrhs) {
  if (!c.bsr && !c.f32) {
    HIP_TRY(launch_residual(c.A->g, c.A->rec64, c.trans, b, x, out, nrhs, c.s));
    return R1S_OK;
  }
  if (int e = op_apply(c, x, out, nrhs)) return e;
  HIP_TRY(launch_rsub(b, out, c.A->g.n, nrhs, c.s));
  return R1S_OK;
}

// Waits until flag[0 .. count) all equal val (flags raised by kernels in
// pinned host memory, see k_dcgs_small / k_stage_flag): a spin instead of an
// event, which would put a barrier between the kernels of consecutive
// steps.  After two seconds it synchronises the stream, after which the
// flags must be set.
static int spin_flags(const int* f, int count, int val, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned it = 1;; ++it) {
    bool ok = true;
    for (int r = 0; r < count && ok; ++r) ok = __atomic_load_n(f + r, __ATOMIC_ACQUIRE) == val;
    if (ok) return R1S_OK;
    if ((it & 4095) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      HIP_TRY(hipStreamSynchronize(s));
      for (int r = 0; r < count; ++r)
        if (__atomic_load_n(f + r, __ATOMIC_ACQUIRE) != val)
          return fail(R1S_ERR_HIP, "staging flag %d not raised after the stream drained", r);
      return R1S_OK;
    }
    __builtin_ia32_pause();
  }
}

// Norms of nrhs contiguous vectors of length n (deterministic, float64).
// |v_r| per right-hand side (|v_r|^2 stays in W.scal); `pinned` (nrhs
// doubles of pinned host memory, or null) receives the device copy, and
// with `flag` (pinned) the host spins on flag[0] == seq instead of
// synchronising the stream.
static int norms(const Mesh& g, GmresWork& W, const double* v, int nrhs, hipStream_t s,
                 std::vector<double>& out, double* pinned = nullptr, int* flag = nullptr,
                 int seq = 0) {
  Basis none{W.V, 0, 0};
  HIP_TRY(launch_multidot(none, 0, v, g.n, g.n, nrhs, W.part, W.nblk, true, s));
  out.assign(nrhs, 0.0);
  double* dst = pinned ? pinned : out.data();
  if (flag && pinned) {  // one kernel reduces, hands the norms over and raises the flag
    HIP_TRY(launch_reduce_host(W.part, nrhs, W.nblk, W.scal, pinned, flag, seq, s));
    if (int e = spin_flags(flag, 1, seq, s)) return e;
  } else {
    HIP_TRY(launch_reduce(W.part, nrhs, W.nblk, W.scal, s));
    HIP_TRY(hipMemcpyAsync(dst, W.scal, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  for (int r = 0; r < nrhs; ++r) out[r] = sqrt(dst[r]);
  return R1S_OK;
}

struct SolveStat {
  int iters = 0, cycles = 0;
  bool converged = false;
  double rel = 0.0;
};

// Restarted right-preconditioned GMRES on nrhs systems op(x) = b, starting
// from x (x0_given) or zero.  rtol is relative to |b| per right-hand side.
// trust_estimate: a cycle whose least-squares residual estimate meets rtol
// for every right-hand side ends the solve without the true residual (for
// the inner solves of iterative refinement, whose caller forms the float64
// residual itself).
// Doubles of one staging slot of the Arnoldi coefficients (all right-hand
// sides): the per-step layout of k_update_normalize or of the delayed
// scheme's k_dcgs_small, whichever is larger.
static size_t stage_slot_doubles(int k, int nrhs) {
  const int HS = k + 2, SS = 2 * k + 6;
  return (size_t)nrhs * std::max(2 * HS + 1, SS);
}

// Where the kernels stage a step's Arnoldi coefficients for the host.  With
// dev == nullptr (r1s_gmres) they write pooled pinned host memory directly
// and an event per slot tells the host when a slot is complete.  Otherwise
// (r1s_gmres_noalloc) they write the two device slots dev[0], dev[1] and the
// host copies a slot into its own memory, synchronising the stream, before
// reading it: one host wait per step instead of none, and nothing allocated.
struct StageDev {
  double* dev[2];
};

static int gmres_core(const OpCtx& c, const Mesh& g, GmresWork& W, int k, int max_cycles,
                      double rtol, int nrhs, const double* b, double* x, bool x0_given,
                      int ortho, bool trust_estimate, std::vector<SolveStat>& st,
                      const StageDev* sd, bool* drained = nullptr) {
  const bool always_reorth = ortho == R1S_ORTHO_CGS2;
  const bool delayed = ortho == R1S_ORTHO_DELAYED;
  hipStream_t s = c.s;
  const long long n = g.n;
  const int HS = k + 2;  // stride of the per-rhs h arrays
  // host staging: two slots of Arnoldi coefficients, then the norms and the
  // least-squares solution of a cycle (pinned, or host copies of the device
  // slots without a pinned pool)
  StagingLease lease;
  lease.stream = s;
  const int SS = 2 * k + 6;  // delayed scheme: staging doubles per right-hand side
  const size_t slot_doubles = stage_slot_doubles(k, nrhs);
  const size_t y_doubles = (size_t)nrhs * (k + 1);
  std::vector<double> host_slots;
  double* stage[2];   // read by the host
  double* kstage[2];  // written by the kernels
  double* pin_norm = nullptr;
  double* pin_y = nullptr;
  // ready flags in pinned memory: [2][nrhs] for the step slots (delayed
  // scheme), one for the norms; zeroed per solve, raised with increasing
  // sequence numbers
  int* pin_flag = nullptr;
  const int nflags = 2 * nrhs + 1;
  if (!sd) {
    const size_t flag_doubles = (size_t)(nflags + 1) / 2;
    if (int e = staging_acquire((2 * slot_doubles + nrhs + y_doubles + flag_doubles) * sizeof(double),
                                &lease.st))
      return e;
    stage[0] = kstage[0] = (double*)lease.st->mem;
    stage[1] = kstage[1] = (double*)lease.st->mem + slot_doubles;
    pin_norm = (double*)lease.st->mem + 2 * slot_doubles;
    pin_y = pin_norm + nrhs;
    pin_flag = (int*)(pin_y + y_doubles);
    for (int i = 0; i < nflags; ++i) __atomic_store_n(pin_flag + i, 0, __ATOMIC_RELAXED);
  } else {
    host_slots.assign(2 * slot_doubles, 0.0);
    stage[0] = host_slots.data();
    stage[1] = host_slots.data() + slot_doubles;
    kstage[0] = sd->dev[0];
    kstage[1] = sd->dev[1];
  }
  // a step's kernels are queued: mark its slot; the host needs a slot: wait.
  // The delayed scheme's steps raise ready flags (want[slot] is the sequence
  // number of the step in the slot); the other schemes record events.
  const bool flags = pin_flag && delayed;
  int seq = 0, want[2] = {0, 0};
  auto step_flag = [&](int slot) -> int* {
    if (!flags) return nullptr;
    want[slot] = ++seq;
    return pin_flag + slot * nrhs;
  };
  auto mark = [&](int slot) -> int {
    if (flags) return R1S_OK;
    if (!sd) {
      HIP_TRY(hipEventRecord(lease.st->ev[slot], s));
    } else {
      HIP_TRY(hipMemcpyAsync(stage[slot], kstage[slot], slot_doubles * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    }
    return R1S_OK;
  };
  auto wait = [&](int slot) -> int {
    if (flags) return spin_flags(pin_flag + slot * nrhs, nrhs, want[slot], s);
    if (!sd) {
      HIP_TRY(hipEventSynchronize(lease.st->ev[slot]));
    } else {
      HIP_TRY(hipStreamSynchronize(s));
    }
    return R1S_OK;
  };
  int* norm_flag = pin_flag ? pin_flag + 2 * nrhs : nullptr;
  std::vector<double> bnorm(nrhs, 0.0);
  st.assign(nrhs, SolveStat());
  // |b| (|b|^2 stays in W.scal).  Starting from zero, the delayed scheme
  // queues the first cycle without it (b_pending): its step 0 normalises b
  // itself and stages |b|^2, which the host takes at the cycle's first wait,
  // so that the device starts with the first step.
  // With it, the first cycle always runs and its update writes x (x = M V y
  // in place of x += M V y), so x needs no clearing.
  const int b_seq = ++seq;
  bool b_pending = !x0_given && delayed;
  const bool x_set_by_update = b_pending;
  if (!x0_given && !b_pending) HIP_TRY(hipMemsetAsync(x, 0, (size_t)nrhs * n * sizeof(double), s));
  if (!b_pending) {
    if (int e = norms(g, W, b, nrhs, s, bnorm, pin_norm, norm_flag, b_seq)) return e;
    for (int r = 0; r < nrhs; ++r)
      if (!(bnorm[r] == bnorm[r]) || isinf(bnorm[r])) return fail(R1S_ERR_NONFINITE, "right-hand side %d is not finite", r);
  }
  // vector-major basis [k + 1][nrhs][n]: v_j of every right-hand side is one
  // contiguous [nrhs][n] block, the layout the operator kernels take
  Basis Vb{W.V, (long long)nrhs * n, n};
  std::vector<double> H((size_t)nrhs * (k + 1) * k), cs((size_t)nrhs * k), sn((size_t)nrhs * k),
      gv((size_t)nrhs * (k + 1)), y((size_t)nrhs * (k + 1)),
      beta, w0(nrhs);
  std::vector<int> jend(nrhs), done(nrhs);
  std::vector<double> est(nrhs, -1.0);  // residual estimate at the end of the last cycle
  auto Hat = [&](int r, int i, int j) -> double& { return H[((size_t)r * (k + 1) + i) * k + j]; };

  for (int cycle = 0;; ++cycle) {
    if (trust_estimate && cycle > 0) {
      bool met = true;
      for (int r = 0; r < nrhs; ++r)
        met = met && (st[r].converged || (est[r] >= 0.0 && est[r] <= rtol * bnorm[r]));
      if (met) {
        for (int r = 0; r < nrhs; ++r) {
          if (st[r].converged) continue;
          st[r].rel = bnorm[r] > 0 ? est[r] / bnorm[r] : 0.0;
          st[r].converged = true;
        }
        break;
      }
    }
    // true residual of the current iterate (x0 = 0: r = b, whose norms are
    // known); the delayed scheme takes it in basis slot 0, which its step 0
    // normalises in place (the operator's output w would overwrite it)
    const bool from_b = cycle == 0 && !x0_given;
    double* rv = delayed ? W.V : W.w;
    if (from_b) {
      beta = bnorm;
    } else {
      if (int e = op_residual(c, b, x, rv, nrhs)) return e;
      if (int e = norms(g, W, rv, nrhs, s, beta, pin_norm, norm_flag, ++seq)) return e;
    }
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      if (b_pending) {  // |b| not known yet: every right-hand side runs (see b_arrived)
        done[r] = 0;
        all = false;
        continue;
      }
      if (!(beta[r] == beta[r]) || isinf(beta[r])) return fail(R1S_ERR_NONFINITE, "residual of right-hand side %d is not finite", r);
      st[r].rel = bnorm[r] > 0 ? beta[r] / bnorm[r] : 0.0;
      st[r].converged = beta[r] <= rtol * bnorm[r];
      done[r] = st[r].converged;
      all = all && done[r];
    }
    if (all || cycle == max_cycles) {
      // the norms just read were the last work queued; with a ready flag the
      // host has seen that kernel's last write, so nothing is left to wait for
      if (pin_flag) {
        lease.drained = true;
        if (drained) *drained = true;
      }
      break;
    }
    for (int r = 0; r < nrhs; ++r) {
      st[r].cycles += done[r] ? 0 : 1;
      jend[r] = 0;
      for (int i = 0; i <= k; ++i) gv[(size_t)r * (k + 1) + i] = 0.0;
      gv[(size_t)r * (k + 1)] = beta[r];
    }
    // the first cycle's |b| has reached the host (called after each wait of
    // the cycle): fill in what the cycle start left open; a zero right-hand
    // side is solved by x = 0 and takes no part in the cycle
    std::vector<char> zero_b(nrhs, 0);
    auto b_arrived = [&]() -> int {  // (step 0's slot is on the host)
      if (!b_pending) return R1S_OK;
      b_pending = false;
      for (int r = 0; r < nrhs; ++r) {
        bnorm[r] = sqrt(stage[0][(size_t)r * SS]);
        if (!(bnorm[r] == bnorm[r]) || isinf(bnorm[r])) return fail(R1S_ERR_NONFINITE, "right-hand side %d is not finite", r);
        beta[r] = bnorm[r];
        gv[(size_t)r * (k + 1)] = beta[r];
        st[r].rel = bnorm[r] > 0 ? 1.0 : 0.0;
        if (bnorm[r] == 0.0) {
          st[r].converged = true;
          st[r].cycles = 0;
          done[r] = 1;
          zero_b[r] = 1;
        }
      }
      return R1S_OK;
    };
    // v_0 = r / |r|, the squared norms still in W.scal from the last norms()
    // (the delayed scheme's step 0 normalises u0 itself)
    const double* u0 = from_b ? b : rv;
    if (!delayed) HIP_TRY(launch_scale_unit(u0, n, W.scal, W.V, Vb.rstride, n, nrhs, s));

    // Givens update of the least-squares problem with column j of H (rows
    // 0..j+1 in Hat): the previous rotations, then a new one eliminating
    // H[j+1][j]; g_{j+1} is then the residual estimate.
    auto givens = [&](int r, int j) {
      for (int i = 0; i < j; ++i) {
        const double a = Hat(r, i, j), bb = Hat(r, i + 1, j);
        Hat(r, i, j) = cs[(size_t)r * k + i] * a + sn[(size_t)r * k + i] * bb;
        Hat(r, i + 1, j) = -sn[(size_t)r * k + i] * a + cs[(size_t)r * k + i] * bb;
      }
      const double a = Hat(r, j, j), bb = Hat(r, j + 1, j);
      const double rho = hypot(a, bb);
      const double cj = rho > 0 ? a / rho : 1.0, sj = rho > 0 ? bb / rho : 0.0;
      cs[(size_t)r * k + j] = cj;
      sn[(size_t)r * k + j] = sj;
      Hat(r, j, j) = rho;
      Hat(r, j + 1, j) = 0.0;
      double* gr = gv.data() + (size_t)r * (k + 1);
      gr[j + 1] = -sj * gr[j];
      gr[j] = cj * gr[j];
      jend[r] = j + 1;
      st[r].iters += 1;
    };
    // Arnoldi steps.  The coefficients of step j reach the host through the
    // pinned staging slot j % 2 while step j + 1 runs on the device; the host
    // updates the least-squares problem of step j only after it has queued
    // step j + 1, so the device never waits for the host.  When step j meets
    // the tolerance, step j + 1 was computed for nothing and is dropped.
    auto process = [&](int j) -> bool {  // true: every right-hand side is done
      const int nv = j + 1;
      const double* h1 = stage[j & 1];  // layout of k_update_normalize's staging
      const double* h2s = h1 + (size_t)nrhs * (nv + 1);
      const double* needs = h2s + (size_t)nrhs * (nv + 1);
      bool all_done = true;
      for (int r = 0; r < nrhs; ++r) {
        if (done[r]) continue;
        const double* h1r = h1 + (size_t)r * (nv + 1);
        const double* h2r = h2s + (size_t)r * (nv + 1);
        const bool two = needs[r] != 0.0;
        const double* hl = two ? h2r : h1r;  // the pass the new vector comes from
        double hh = 0.0;
        for (int i = 0; i < nv; ++i) {
          Hat(r, i, j) = h1r[i] + (two ? h2r[i] : 0.0);
          hh += hl[i] * hl[i];
        }
        const double q = hl[nv] - hh;
        const double hn = q > 0.0 ? sqrt(q) : 0.0;
        const double wnorm0 = sqrt(h1r[nv]);
        Hat(r, j + 1, j) = hn;
        givens(r, j);
        const bool breakdown = hn <= 1e-14 * wnorm0;
        if (breakdown || fabs(gv[(size_t)r * (k + 1) + j + 1]) <= rtol * bnorm[r]) done[r] = 1;
        all_done = all_done && done[r];
      }
      return all_done;
    };
    if (delayed) {
      // One reduction per step (device kernels k_dcgs_*): step j turns the
      // lagged u_j in slot j into the final v_j, finalises column j - 1 of H
      // and estimates column j; the host takes the final columns for the
      // least-squares problem and tests the estimated one for convergence.
      // lastcol[r]: the last column of right-hand side r once it has met the
      // tolerance (or broken down) on an estimated column, else -1.
      std::vector<int> lastcol(nrhs, -1);
      for (int r = 0; r < nrhs; ++r)
        if (done[r]) lastcol[r] = -2;  // converged before this cycle: nothing to do
      auto final_col = [&](int j, const double* stg) {  // column j, staged by step j + 1
        for (int r = 0; r < nrhs; ++r) {
          if (lastcol[r] == -2 || (lastcol[r] >= 0 && j > lastcol[r])) continue;
          const double* h = stg + (size_t)r * SS;
          for (int i = 0; i <= j + 1; ++i) Hat(r, i, j) = h[i];
          givens(r, j);
        }
      };
      std::vector<double> col(k + 2);
      auto trial = [&](int j, const double* stg) {  // estimated column j, staged by step j
        for (int r = 0; r < nrhs; ++r) {
          if (lastcol[r] != -1) continue;
          const double* h = stg + (size_t)r * SS;
          for (int i = 0; i <= j; ++i) col[i] = h[k + 1 + i];
          col[j + 1] = h[2 * k + 2];
          for (int i = 0; i < j; ++i) {
            const double a = col[i], bb = col[i + 1];
            col[i] = cs[(size_t)r * k + i] * a + sn[(size_t)r * k + i] * bb;
            col[i + 1] = -sn[(size_t)r * k + i] * a + cs[(size_t)r * k + i] * bb;
          }
          const double rho = hypot(col[j], col[j + 1]);
          const double sj = rho > 0 ? col[j + 1] / rho : 0.0;
          const double res = fabs(sj * gv[(size_t)r * (k + 1) + j]);
          const bool breakdown = h[2 * k + 2] <= 1e-14 * h[2 * k + 3] || h[2 * k + 5] != 0.0;
          if (breakdown || res <= rtol * bnorm[r]) lastcol[r] = j;
        }
      };
      auto launch_step = [&](int j) -> int {
        if (int e = prec_apply(c, j == 0 ? u0 : W.V + (long long)j * Vb.vstride, W.z, nrhs))
          return e;
        if (int e = op_apply(c, W.z, W.w, nrhs)) return e;
        HIP_TRY(launch_dcgs_dots(Vb, j, u0, n, W.w, n, n, nrhs, W.part, W.nblk, s));
        int* fl = step_flag(j & 1);
        HIP_TRY(launch_dcgs_small(j, k, W.part, W.nblk, W.dstate, W.dstride, kstage[j & 1], SS,
                                  false, nrhs, s, fl, want[j & 1]));
        HIP_TRY(launch_dcgs_update(Vb, j, k, W.dstate, W.dstride, u0, n, W.w, n, n, nrhs, s));
        return mark(j & 1);
      };
      auto all_stopped = [&]() {
        for (int r = 0; r < nrhs; ++r)
          if (lastcol[r] == -1) return false;
        return true;
      };
      // after each wait: the first cycle's |b| (a zero right-hand side stops)
      auto arrived = [&]() -> int {
        const bool was = b_pending;
        if (int e = b_arrived()) return e;
        if (was)
          for (int r = 0; r < nrhs; ++r)
            if (zero_b[r]) lastcol[r] = -2;
        return R1S_OK;
      };
      bool stopped = false;
      for (int j = 0; j < k && !stopped; ++j) {
        if (int e = launch_step(j)) return e;
        if (j == 0) continue;
        if (int e = wait((j - 1) & 1)) return e;
        if (int e = arrived()) return e;
        if (j >= 2) final_col(j - 2, stage[(j - 1) & 1]);
        trial(j - 1, stage[(j - 1) & 1]);
        if (all_stopped()) {  // the final column j - 1 comes from step j
          if (int e = wait(j & 1)) return e;
          final_col(j - 1, stage[j & 1]);
          stopped = true;
        }
      }
      if (!stopped) {
        // the cycle's last step k - 1: its final column needs one more
        // reduction on u_k (slot k), without the operator
        if (int e = wait((k - 1) & 1)) return e;
        if (int e = arrived()) return e;
        if (k >= 2) final_col(k - 2, stage[(k - 1) & 1]);
        trial(k - 1, stage[(k - 1) & 1]);
        const double* uk = W.V + (long long)k * Vb.vstride;
        HIP_TRY(launch_dcgs_dots(Vb, k, nullptr, 0, uk, Vb.rstride, n, nrhs, W.part, W.nblk, s));
        int* fl = step_flag(k & 1);
        HIP_TRY(launch_dcgs_small(k, k, W.part, W.nblk, W.dstate, W.dstride, kstage[k & 1], SS,
                                  true, nrhs, s, fl, want[k & 1]));
        if (int e = mark(k & 1)) return e;
        if (int e = wait(k & 1)) return e;
        final_col(k - 1, stage[k & 1]);
      }
      for (int r = 0; r < nrhs; ++r)
        if (lastcol[r] == -2) jend[r] = 0;
    }
    int pending = -1;  // step whose coefficients are staged but not yet used
    bool finished = delayed;
    for (int j = 0; j < k && !delayed; ++j) {
      // z = M v_j ; w = op(z)
      if (int e = prec_apply(c, W.V + (long long)j * Vb.vstride, W.z, nrhs)) return e;
      if (int e = op_apply(c, W.z, W.w, nrhs)) return e;
      const int nv = j + 1;
      // Classical Gram-Schmidt: h1 = V^T w and |w|^2 in one pass.  The norm
      // of w - V h1 follows from |w|^2 - |h1|^2 (V orthonormal); a second
      // pass (reorthogonalisation) runs where that norm dropped below |w| /
      // sqrt(2) (Daniel-Gragg-Kaufman-Stewart criterion, decided on the
      // device per right-hand side), or on every step with always_reorth or
      // a basis of more than 16 vectors.
      // (h1, h2: rows of nv + 1 values per rhs)
      double* h2 = W.hdev + (size_t)nrhs * HS;
      HIP_TRY(launch_multidot(Vb, nv, W.w, n, n, nrhs, W.part, W.nblk, true, s));
      HIP_TRY(launch_reduce(W.part, nrhs * (nv + 1), W.nblk, W.hdev, s));
      const bool fused = nv <= update_multidot_max();
      if (fused) {  // w -= V h1 and V^T w in one pass, where needed
        HIP_TRY(launch_update_multidot(Vb, nv, W.hdev, nv + 1, W.w, n, n, nrhs, W.part, W.nblk,
                                       always_reorth, W.need, s));
      } else {
        HIP_TRY(launch_update(Vb, nv, W.hdev, nv + 1, W.w, n, n, nrhs, s));
        HIP_TRY(launch_multidot(Vb, nv, W.w, n, n, nrhs, W.part, W.nblk, true, s));
      }
      HIP_TRY(launch_reduce(W.part, nrhs * (nv + 1), W.nblk, h2, s));
      // v_{j+1} = (w - V h) / |w - V h| with h the last pass's coefficients;
      // the coefficients go to the host staging slot of this step
      const int slot = j & 1;
      HIP_TRY(launch_update_normalize(Vb, nv, W.hdev, h2, nv + 1, fused ? W.need : nullptr, W.w,
                                      n, W.V + (long long)(j + 1) * Vb.vstride, n, nrhs, s,
                                      kstage[slot]));
      if (int e = mark(slot)) return e;
      if (pending >= 0) {
        if (int e = wait(pending & 1)) return e;
        const bool all_done = process(pending);
        pending = -1;
        if (all_done) {
          finished = true;
          break;
        }
      }
      pending = j;
    }
    if (!finished && pending >= 0) {  // (not reached in the delayed scheme)
      if (int e = wait(pending & 1)) return e;
      process(pending);
    }
    if (int e = b_arrived()) return e;  // (done by the first wait of the cycle)
    // y = R^{-1} g per rhs; x += M (V y)
    std::fill(y.begin(), y.end(), 0.0);
    for (int r = 0; r < nrhs; ++r) {
      const int je = jend[r];
      double* yr = y.data() + (size_t)r * (k + 1);
      const double* gr = gv.data() + (size_t)r * (k + 1);
      for (int i = je - 1; i >= 0; --i) {
        double acc = gr[i];
        for (int l = i + 1; l < je; ++l) acc -= Hat(r, i, l) * yr[l];
        yr[i] = Hat(r, i, i) != 0.0 ? acc / Hat(r, i, i) : 0.0;
      }
      if (!st[r].converged) est[r] = fabs(gr[je]);  // |g_je| after the rotations
    }
    int kmax = 0;
    for (int r = 0; r < nrhs; ++r) kmax = std::max(kmax, jend[r]);
    if ((long long)nrhs * kmax <= COMBINE_Y_MAX) {  // y passed with the launch
      HIP_TRY(launch_combine_arg(Vb, kmax, y.data(), k + 1, W.t, n, n, nrhs, s));
    } else {
      // (the next cycle's norms synchronise before pin_y is written again; a
      // copy from pageable memory has taken the data when it returns)
      if (pin_y) std::copy(y.begin(), y.end(), pin_y);
      HIP_TRY(hipMemcpyAsync(W.ydev, pin_y ? pin_y : y.data(), y.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
      HIP_TRY(launch_combine(Vb, kmax, W.ydev, k + 1, W.t, n, n, nrhs, s));
    }
    if (cycle == 0 && x_set_by_update) {
      if (int e = prec_apply(c, W.t, x, nrhs)) return e;
    } else {
      if (int e = prec_apply(c, W.t, W.z, nrhs)) return e;
      HIP_TRY(launch_axpy(nullptr, W.z, x, n, nrhs, s));
    }
  }
  return R1S_OK;
}

// Argument checks shared by r1s_gmres and r1s_gmres_noalloc.
static int gmres_check(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts, int nrhs,
                       const double* b, const double* x) {
  if (!A || !M) return fail(R1S_ERR_ARG, "matrix or preconditioner handle is NULL");
  if (int e = check_opts(opts)) return e;
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  if (int e = check_vec(b, "b")) return e;
  if (int e = check_vec(x, "x")) return e;
  if (b == x) return fail(R1S_ERR_ARG, "b and x must not alias");
  if (opts->op == R1S_OP_BSR && !B) return fail(R1S_ERR_ARG, "BSR operator requested but B is NULL");
  if (opts->op == R1S_OP_BSR && opts->trans) return fail(R1S_ERR_UNSUPPORTED, "BSR operator: no transposed solve");
  if (B && (B->g.nx != A->g.nx || B->g.ny != A->g.ny || B->g.L != A->g.L))
    return fail(R1S_ERR_ARG, "BSR handle does not match the matrix");
  if (M->g.nx != A->g.nx || M->g.ny != A->g.ny || M->g.L != A->g.L)
    return fail(R1S_ERR_ARG, "preconditioner does not match the matrix");
  if (M->g.rd != A->g.rd || M->g.ro != A->g.ro || M->g.band != A->g.band ||
      M->g.arrow != A->g.arrow || M->g.pat != A->g.pat || M->g.pnnz != A->g.pnnz)
    return fail(R1S_ERR_ARG, "preconditioner was set up for another block layout");
  if (opts->trans && M->kind == PREC_SMW && !smw_has_trans(M))
    return fail(R1S_ERR_ARG, "transposed solve needs a preconditioner set up with R1S_WITH_TRANS");
  if (opts->trans && M->kind == PREC_BSR_LU)
    return fail(R1S_ERR_UNSUPPORTED, "dense-LU preconditioner: no transposed apply");
  const bool mixed = opts->mode == R1S_MODE_MIXED_IR;
  if (mixed && (!A->rec32 || M->kind != PREC_SMW || !smw_has_f32(M)))
    return fail(R1S_ERR_ARG, "mixed mode needs R1S_KEEP_F32 on the matrix and the preconditioner");
  return R1S_OK;
}

// The solve itself (arguments checked, W carved from the workspace).
static int gmres_run(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts, int nrhs,
                     const double* b, double* x, GmresWork& W, const StageDev* sd,
                     r1s_gmres_stats* stats, hipStream_t s) {
  const Mesh& g = A->g;
  const bool mixed = opts->mode == R1S_MODE_MIXED_IR;
  OpCtx c{A, B, M, false, opts->trans != 0, opts->op == R1S_OP_BSR, s};
  std::vector<SolveStat> st;
  int outer = 0;
  int rc;
  bool drained = false;
  if (!mixed) {
    rc = gmres_core(c, g, W, opts->restart, opts->max_cycles, opts->rtol, nrhs, b, x,
                    opts->x0_given != 0, opts->ortho, false, st, sd, &drained);
    if (rc) return rc;
  } else {
    // iterative refinement: r = b - J x (float64), inner float32 solve J d = r
    // (from x = 0 the first residual is b, and the first correction is x)
    std::vector<double> bnorm, rn;
    StagingLease nlease;  // pinned landing buffer of the outer norms (r1s_gmres)
    nlease.stream = s;
    double* pin_norm = nullptr;
    if (!sd) {
      if (int e = staging_acquire((size_t)nrhs * sizeof(double), &nlease.st)) return e;
      pin_norm = (double*)nlease.st->mem;
    }
    if (int e = norms(g, W, b, nrhs, s, bnorm, pin_norm)) return e;
    const bool zero_start = !opts->x0_given;
    OpCtx ci = c;
    ci.f32 = true;
    std::vector<SolveStat> tot(nrhs);
    for (;; ++outer) {
      const bool first = outer == 0 && zero_start;
      if (first) {
        rn = bnorm;
      } else {
        if (int e = op_residual(c, b, x, W.r64, nrhs)) return e;
        if (int e = norms(g, W, W.r64, nrhs, s, rn, pin_norm)) return e;
      }
      bool all = true;
      for (int r = 0; r < nrhs; ++r) {
        if (!(rn[r] == rn[r]) || isinf(rn[r])) return fail(R1S_ERR_NONFINITE, "refinement residual %d is not finite", r);
        tot[r].rel = bnorm[r] > 0 ? rn[r] / bnorm[r] : 0.0;
        tot[r].converged = rn[r] <= opts->rtol * bnorm[r];
        all = all && tot[r].converged;
      }
      if (all || outer == opts->max_outer) {
        if (first) HIP_TRY(hipMemsetAsync(x, 0, (size_t)nrhs * g.n * sizeof(double), s));
        break;
      }
      std::vector<SolveStat> in;
      rc = gmres_core(ci, g, W, opts->restart, opts->max_cycles, opts->inner_rtol, nrhs,
                      first ? b : W.r64, first ? x : W.d, false, opts->ortho, true, in, sd);
      if (rc) return rc;
      for (int r = 0; r < nrhs; ++r) {
        tot[r].iters += in[r].iters;
        tot[r].cycles += in[r].cycles;
      }
      if (!first) HIP_TRY(launch_axpy(nullptr, W.d, x, g.n, nrhs, s));
    }
    st = tot;
  }
  if (!drained) HIP_TRY(hipStreamSynchronize(s));
  bool ok = true;
  for (int r = 0; r < nrhs; ++r) {
    ok = ok && st[r].converged;
    if (stats) {
      stats[r].iters = st[r].iters;
      stats[r].cycles = st[r].cycles;
      stats[r].outer = outer;
      stats[r].converged = st[r].converged ? 1 : 0;
      stats[r].rel_residual = st[r].rel;
    }
  }
  if (!ok) return fail(R1S_ERR_NOCONV, "GMRES did not reach rtol %g", opts->rtol);
  return R1S_OK;
}

extern "C" int r1s_gmres(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts, int nrhs,
                         const double* b, double* x, void* work, size_t work_bytes,
                         r1s_gmres_stats* stats, void* stream) {
  if (int e = gmres_check(A, B, M, opts, nrhs, b, x)) return e;
  if (!work || !aligned(work, 256)) return fail(R1S_ERR_ARG, "work is NULL or not 256-byte aligned");
  size_t need;
  if (int e = r1s_gmres_work_size(A, opts, nrhs, &need)) return e;
  if (work_bytes < need) return fail(R1S_ERR_ARG, "work_bytes %zu < required %zu", work_bytes, need);
  GmresWork W;
  Carver cv(work);
  gmres_layout(cv, A->g, opts->restart, nrhs, opts->mode == R1S_MODE_MIXED_IR, &W);
  return gmres_run(A, B, M, opts, nrhs, b, x, W, nullptr, stats, as_stream(stream));
}

// ------------------------------------------------- GMRES without allocation --
// The workspace of r1s_gmres_noalloc: one array per GPU for the life of the
// process.  Host code never passes its name to a kernel or a copy (in host
// code it is a stand-in, not a device address): scratch_ptr() gives each
// device's own copy, looked up once per device.
static __device__ __align__(256) unsigned char scratch[R1S_NOALLOC_MAX_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[64];  // per device id, set on first use

static int scratch_ptr(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(R1S_ERR_UNSUPPORTED, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(R1S_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return R1S_OK;
}

// Bytes of the static workspace a solve takes: r1s_gmres's workspace and the
// two device staging slots.
static int noalloc_bytes(r1s_mat A, const r1s_gmres_opts* opts, int nrhs, size_t* bytes) {
  size_t need;
  if (int e = r1s_gmres_work_size(A, opts, nrhs, &need)) return e;
  const size_t slot = (stage_slot_doubles(opts->restart, nrhs) * sizeof(double) + 255) & ~(size_t)255;
  *bytes = ((need + 255) & ~(size_t)255) + 2 * slot;
  return R1S_OK;
}

extern "C" int r1s_gmres_noalloc_size(r1s_mat A, const r1s_gmres_opts* opts, int nrhs,
                                      size_t* bytes) {
  if (!A || !bytes) return fail(R1S_ERR_ARG, "NULL argument");
  if (int e = check_opts(opts)) return e;
  if (nrhs < 1) return fail(R1S_ERR_ARG, "nrhs must be >= 1");
  return noalloc_bytes(A, opts, nrhs, bytes);
}

extern "C" int r1s_gmres_noalloc(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts,
                                 int nrhs, const double* b, double* x, r1s_gmres_stats* stats,
                                 void* stream) {
  if (int e = gmres_check(A, B, M, opts, nrhs, b, x)) return e;
  size_t need;
  if (int e = noalloc_bytes(A, opts, nrhs, &need)) return e;
  if (need > (size_t)R1S_NOALLOC_MAX_BYTES)
    return fail(R1S_ERR_ARG,
                "the solve needs %zu bytes of workspace, more than the %llu of r1s_gmres_noalloc "
                "(use r1s_gmres with a caller-owned workspace)",
                need, (unsigned long long)R1S_NOALLOC_MAX_BYTES);
  void* base = nullptr;
  if (int e = scratch_ptr(&base)) return e;
  GmresWork W;
  Carver cv(base);
  gmres_layout(cv, A->g, opts->restart, nrhs, opts->mode == R1S_MODE_MIXED_IR, &W);
  const size_t slot = stage_slot_doubles(opts->restart, nrhs);
  StageDev sd;
  sd.dev[0] = cv.take<double>(slot);
  sd.dev[1] = cv.take<double>(slot);
  return gmres_run(A, B, M, opts, nrhs, b, x, W, &sd, stats, as_stream(stream));
}

// ------------------------------------------------------------ gradients ---
extern "C" int r1s_grad(r1s_mat A, int nrhs, const double* lambda, const double* x,
                        const r1s_grads* out, void* stream) {
  if (!A || !out) return fail(R1S_ERR_ARG, "NULL argument");
  if (A->g.graph) return fail(R1S_ERR_ARG, "general-mesh matrix: use r1s_grad_graph");
  if (A->g.pat) return fail(R1S_ERR_ARG, "general-pattern matrix: use r1s_grad_pattern");
  if (nrhs < 1 || nrhs > 64) return fail(R1S_ERR_ARG, "nrhs must be in [1, 64]");
  if (int e = check_vec(lambda, "lambda")) return e;
  if (int e = check_vec(x, "x")) return e;
  const Mesh& g = A->g;
  const void* ps[10] = {out->s_diag, out->s_sub, out->s_sup, out->s_flow, out->s_nbr,
                        out->u,      out->v,     out->s_band, out->s_lev_flow, out->s_flow_lev};
  const bool used[10] = {true, g.L > 1, g.L > 1, true, true, true, true,
                         g.band > 1, g.arrow != 0, g.arrow != 0};
  for (int i = 0; i < 10; ++i) {
    if (!used[i]) continue;
    if (int e = check_vec(ps[i], "gradient output")) return e;
  }
  GradOut o{out->s_diag, out->s_sub, out->s_sup, out->s_flow, out->s_nbr, out->u, out->v,
            out->s_band, out->s_lev_flow, out->s_flow_lev};
  HIP_TRY(launch_grad(A->g, A->rec64, lambda, x, nrhs, o, as_stream(stream)));
  return R1S_OK;
}

extern "C" int r1s_grad_pattern(r1s_mat A, int nrhs, const double* lambda, const double* x,
                                const r1s_pattern_grads* out, void* stream) {
  if (!A || !out) return fail(R1S_ERR_ARG, "NULL argument");
  if (!A->g.pat) return fail(R1S_ERR_ARG, "not a general-pattern matrix: use r1s_grad");
  if (nrhs < 1 || nrhs > 64) return fail(R1S_ERR_ARG, "nrhs must be in [1, 64]");
  if (int e = check_vec(lambda, "lambda")) return e;
  if (int e = check_vec(x, "x")) return e;
  const void* ps[4] = {out->s_cc, out->s_nbr, out->u, out->v};
  for (int i = 0; i < 4; ++i)
    if (int e = check_vec(ps[i], "gradient output")) return e;
  GradOut o{};
  o.s_cc = out->s_cc;
  o.s_nbr = out->s_nbr;
  o.u = out->u;
  o.v = out->v;
  HIP_TRY(launch_grad(A->g, A->rec64, lambda, x, nrhs, o, as_stream(stream)));
  return R1S_OK;
}

extern "C" int r1s_grad_graph(r1s_mat A, int nrhs, const double* lambda, const double* x,
                              const r1s_graph_grads* out, void* stream) {
  if (!A || !out) return fail(R1S_ERR_ARG, "NULL argument");
  if (!A->g.graph) return fail(R1S_ERR_ARG, "structured-mesh matrix: use r1s_grad");
  if (nrhs < 1 || nrhs > 64) return fail(R1S_ERR_ARG, "nrhs must be in [1, 64]");
  if (int e = check_vec(lambda, "lambda")) return e;
  if (int e = check_vec(x, "x")) return e;
  const Mesh& g = A->g;
  const long long n_off = mat_blocks(A) - g.N;
  const void* ps[12] = {out->s_diag, out->s_sub, out->s_sup, out->s_flow, out->s_band,
                        out->s_lev_flow, out->s_flow_lev, out->s_nbr, out->u_diag, out->v_diag,
                        out->u_off, out->v_off};
  const bool used[12] = {true, g.L > 1, g.L > 1, true, g.band > 1, g.arrow != 0, g.arrow != 0,
                         n_off > 0, true, true, n_off > 0 && g.ro > 0, n_off > 0 && g.ro > 0};
  for (int i = 0; i < 12; ++i) {
    if (!used[i]) continue;
    if (int e = check_vec(ps[i], "gradient output")) return e;
  }
  GraphGradOut o{out->s_diag, out->s_sub, out->s_sup, out->s_flow, out->s_band, out->s_lev_flow,
                 out->s_flow_lev, out->s_nbr, out->u_diag, out->v_diag, out->u_off, out->v_off};
  HIP_TRY(launch_grad_graph(g, A->rec64, lambda, x, nrhs, o, as_stream(stream)));
  return R1S_OK;
}
