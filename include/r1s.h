/*
 * r1s -- block r1-sparse Jacobians on MI355X (gfx950).
 *
 * C ABI of libr1s.so.  The Jacobian of a first-order finite-volume
 * discretisation on a structured nx x ny mesh (5-point block stencil, blocks
 * of size m = L + 3: L level densities, two momenta, energy) is held as a
 * fully sparse matrix S plus rank-one pairs per block, the "block r1-sparse"
 * representation of section 4 (Overall Structure) and section 5.1 (BR1-BSR
 * format, where the pair count differs between diagonal and off-diagonal
 * blocks):
 *
 *     J = S + sum over blocks (c, d) of  sum_p u_{c,d,p} v_{c,d,p}^T .
 *
 * Every diagonal block carries r_diag pairs and every neighbour block r_off
 * (section 4, Overall Structure: 9 and 2 for the state-to-state model, one
 * temporal-source pair plus two per trace flux; 1 and 1 is the smallest
 * layout).  Supported: 1 <= r_diag <= 9, 0 <= r_off <= 6 (an HLL flux
 * Jacobian in primitive variables puts the non-diagonal sparse entries of a
 * neighbour block into four more exact pairs: 2 + 4 = 6).
 *
 * The sparse diagonal block S_{c,C} has a level band of half-width `band`
 * (section 4, Temporal Source Jacobian: level-changing processes up to a
 * threshold jump give a banded pattern; band = 1 is tridiagonal) and, with
 * `arrow`, dense coupling of the level rows to the three flow columns
 * (temperature dependence of the level sources) and of the flow rows to the
 * levels.  With arrow = 2 the last level a = L - 1 is the atom density, and
 * the dissociation-recombination processes of the same passage couple it to
 * every molecule level: a dense atom column S_{c,C}[k][a] and atom row
 * S_{c,C}[a][k], k < a, are added to the block (on top of any band entry at
 * those positions).  These are described by r1s_layout; a NULL layout means
 * one pair per block, band = 1, no coupling.
 *
 * The library multiplies by J and J^T (section 5.2), applies the block-Jacobi
 * preconditioner through the Sherman-Morrison-Woodbury identity (section 6,
 * eq. SMW, with the sign of the correction term corrected to minus), and
 * solves J x = b by restarted right-preconditioned GMRES (section 6, eq.
 * right_precond_system).  A dense-block BSR representation of the same J
 * (section 3, Jacobian Complexity; section 5.1, BSR format) with dense-LU
 * block-Jacobi is provided as the baseline.
 *
 * Conventions
 * -----------
 * - Every call returns an int status (R1S_OK = 0, negative on error) and
 *   never throws.  r1s_last_error() returns a thread-local message for the
 *   last failing call on the calling thread.
 * - Arguments are validated on the host before any device work is issued; a
 *   call that fails validation has no side effect.
 * - All device memory is owned by the caller.  *_size calls report how many
 *   bytes a buffer must have; the caller passes a device buffer of at least
 *   that size (256-byte aligned) to the matching *_init / *_setup call and
 *   keeps it alive while the handle is in use.  Handles are small host
 *   objects created by *_init / *_setup and released by *_destroy; they do
 *   not own the device buffer.  The library never keeps a pointer to a
 *   user input buffer after the call that received it returns.
 * - `stream` is a hipStream_t (NULL = the null stream).  Matvec, apply and
 *   grad calls are asynchronous on that stream.  *_init, *_setup and
 *   r1s_gmres synchronise the stream before returning.
 * - Handles are not thread-safe; calls that use one handle must be ordered.
 * - Vectors are float64, C-contiguous, shape [nrhs][N][m] (N = nx*ny cells,
 *   cell c = iy*nx + ix, unknown g = c*m + k), device pointers, 8-byte
 *   aligned.  Input and output vectors must not overlap.
 *
 * Structured input layout (device pointers, float64, C-contiguous)
 * ----------------------------------------------------------------
 *   s_diag [N][m]     diagonal of S_{c,C}
 *   s_sub  [N][L-1]   S_{c,C}[k+1][k], the level band below the diagonal
 *   s_sup  [N][L-1]   S_{c,C}[k][k+1], the level band above the diagonal
 *   s_flow [N][6]     flow-corner off-diagonals of S_{c,C} (rows/columns
 *                     L..L+2) in the order (0,1) (0,2) (1,0) (1,2) (2,0) (2,1)
 *   s_nbr  [N][4][m]  diagonals of the neighbour blocks S_{c,d}, d = S,W,E,N
 *   u, v   [N][P][m]  rank-one pairs, P = r_diag + 4 r_off, in block order
 *                     S (r_off slots), W (r_off), C (r_diag), E (r_off),
 *                     N (r_off)
 *   s_band [N][2(band-1)][L]  (band > 1) level diagonals j = 2..band: row
 *                     j-2 holds S_{c,C}[k][k-j], row band-1+j-2 holds
 *                     S_{c,C}[k][k+j], both at index k (entries outside the
 *                     block must be finite and are ignored)
 *   s_lev_flow [N][ns][L]  (arrow) S_{c,C}[k][L+i] at [c][i][k], i < 3;
 *                     arrow = 2 (ns = 4): slot 3 holds the atom column
 *                     S_{c,C}[k][a] at [c][3][k], k < a
 *   s_flow_lev [N][ns][L]  (arrow) S_{c,C}[L+i][k] at [c][i][k], i < 3;
 *                     arrow = 2: slot 3 holds the atom row S_{c,C}[a][k]
 *                     ns = 3 for arrow = 1, 4 for arrow = 2; index a of slot
 *                     3 must be finite and is ignored
 * Directions: S = (ix, iy-1), W = (ix-1, iy), C = the cell, E = (ix+1, iy),
 * N = (ix, iy+1).  The mesh is not periodic: slots of blocks that do not
 * exist must hold finite values and are treated as zero.  s_sub / s_sup may
 * be NULL when L = 1; s_band, s_lev_flow, s_flow_lev may be NULL when the
 * layout does not use them.
 */
#ifndef R1S_H
#define R1S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status --- */
#define R1S_OK 0
#define R1S_ERR_ARG (-1)         /* invalid argument (dims, pointer, size)  */
#define R1S_ERR_ALLOC (-2)       /* host allocation failed                   */
#define R1S_ERR_HIP (-3)         /* a HIP runtime call failed                */
#define R1S_ERR_SINGULAR (-4)    /* zero pivot or singular SMW capacitance   */
#define R1S_ERR_NOCONV (-5)      /* GMRES did not reach the tolerance        */
#define R1S_ERR_NONFINITE (-6)   /* NaN or Inf met in a residual             */
#define R1S_ERR_UNSUPPORTED (-7) /* valid but unsupported (e.g. m > 256)     */

/* ------------------------------------------------------------- flags --- */
#define R1S_F64 0 /* precision argument: float64 values, float64 arithmetic */
#define R1S_F32 1 /* float32 values and accumulation, float64 vectors       */

#define R1S_KEEP_F32 1   /* also keep float32 copies (mixed precision)      */
#define R1S_WITH_TRANS 2 /* preconditioner: also set up the transposed apply */

#define R1S_MAX_M 256   /* largest supported block size m = L + 3 */
#define R1S_MAX_BAND 8  /* largest level-band half-width of S_{c,C} */
#define R1S_MAX_NBR 8   /* general mesh: most off-diagonal blocks in a block row */

typedef struct r1s_mat_s* r1s_mat;   /* structured r1-sparse Jacobian      */
typedef struct r1s_prec_s* r1s_prec; /* block-Jacobi preconditioner        */
typedef struct r1s_bsr_s* r1s_bsr;   /* dense-block BSR copy of a Jacobian */

/* Block structure of the Jacobian (see the layout above). */
typedef struct {
  int r_diag; /* rank-one pairs per diagonal block, 1..9          */
  int r_off;  /* rank-one pairs per neighbour block, 0..6         */
  int band;   /* level-band half-width of S_{c,C}, 1..R1S_MAX_BAND */
  int arrow;  /* 1: level rows x flow columns, flow rows x levels;
                 2: also the atom (level L-1) x every level        */
} r1s_layout;

typedef struct {
  const double* s_diag;
  const double* s_sub;
  const double* s_sup;
  const double* s_flow;
  const double* s_nbr;
  const double* u;
  const double* v;
  const double* s_band;
  const double* s_lev_flow;
  const double* s_flow_lev;
} r1s_inputs;

/* Gradient outputs, same shapes as r1s_inputs (device pointers, written;
 * the last three only for layouts that have them). */
typedef struct {
  double* s_diag;
  double* s_sub;
  double* s_sup;
  double* s_flow;
  double* s_nbr;
  double* u;
  double* v;
  double* s_band;
  double* s_lev_flow;
  double* s_flow_lev;
} r1s_grads;

/* Inputs on a general mesh (r1s_mat_init_graph).  Per cell, the diagonal
 * block as on the structured mesh: s_diag [N][m], s_sub, s_sup [N][L-1],
 * s_flow [N][6], s_band / s_lev_flow / s_flow_lev (layouts that use them),
 * its r_diag pairs u_diag, v_diag [N][r_diag][m].  Per off-diagonal block, in
 * the order of block_indices with each row's diagonal entry skipped: its
 * diagonal s_nbr [n_off][m] and r_off pairs u_off, v_off [n_off][r_off][m]. */
typedef struct {
  const double* s_diag;
  const double* s_sub;
  const double* s_sup;
  const double* s_flow;
  const double* s_band;
  const double* s_lev_flow;
  const double* s_flow_lev;
  const double* s_nbr;
  const double* u_diag;
  const double* v_diag;
  const double* u_off;
  const double* v_off;
} r1s_graph_inputs;

/* Inputs with a general pattern of S_{c,C} (r1s_mat_init_pattern): s_cc
 * [N][nnz], the values of the pattern's entries in its entry order; s_nbr,
 * u, v as in r1s_inputs. */
typedef struct {
  const double* s_cc;
  const double* s_nbr;
  const double* u;
  const double* v;
} r1s_pattern_inputs;

/* Gradient outputs with a general pattern, same shapes as
 * r1s_pattern_inputs. */
typedef struct {
  double* s_cc;
  double* s_nbr;
  double* u;
  double* v;
} r1s_pattern_grads;

/* Gradient outputs on a general mesh, same shapes as r1s_graph_inputs. */
typedef struct {
  double* s_diag;
  double* s_sub;
  double* s_sup;
  double* s_flow;
  double* s_band;
  double* s_lev_flow;
  double* s_flow_lev;
  double* s_nbr;
  double* u_diag;
  double* v_diag;
  double* u_off;
  double* v_off;
} r1s_graph_grads;

typedef struct {
  int64_t n_cells, n_blocks, m;
  int64_t structured_values;  /* algorithmic stored values of S + u/v      */
  int64_t structured_padded;  /* values actually held (64-byte row padding) */
  int64_t bsr_values;         /* B * m^2 of the dense-block representation */
  int64_t index_bytes;        /* explicit index data: 0 on the structured
                                 mesh; the int32 slot tables on a general one */
  int64_t matvec_bytes;       /* algorithmic HBM bytes of one F64 matvec   */
  int64_t smw_apply_bytes;    /* algorithmic HBM bytes of one F64 apply    */
} r1s_storage;

/* GMRES operator / mode selectors. */
#define R1S_OP_STRUCTURED 0
#define R1S_OP_BSR 1
#define R1S_MODE_F64 0      /* float64 operator and preconditioner          */
#define R1S_MODE_MIXED_IR 1 /* float32 inner GMRES operator + preconditioner,
                               float64 Arnoldi, residual and refinement     */

typedef struct {
  int restart;      /* Krylov space size per cycle (k of GMRES(k)), >= 1   */
  int max_cycles;   /* restart cycles per (inner) solve                     */
  double rtol;      /* stop when |b - J x|_2 <= rtol |b|_2 (per right-hand side) */
  int trans;        /* 1: solve J^T x = b (needs R1S_WITH_TRANS)            */
  int x0_given;     /* 1: x holds the initial guess; 0: start from zero     */
  int op;           /* R1S_OP_STRUCTURED or R1S_OP_BSR                      */
  int mode;         /* R1S_MODE_F64 or R1S_MODE_MIXED_IR                    */
  double inner_rtol;/* mixed mode: relative tolerance of each inner solve   */
  int max_outer;    /* mixed mode: iterative-refinement steps               */
  int ortho;        /* Arnoldi orthogonalisation, R1S_ORTHO_*             */
} r1s_gmres_opts;

/* Orthogonalisation of the Arnoldi vectors (all classical Gram-Schmidt with
 * a second pass, float64): */
#define R1S_ORTHO_DELAYED 0   /* second pass delayed to the next step and
                                 merged with its first: one reduction and
                                 two passes over the basis per step (the
                                 fastest; a zeroed r1s_gmres_opts selects it) */
#define R1S_ORTHO_SELECTIVE 1 /* second pass where |w - V h| < |w| / sqrt(2)
                                 (decided per right-hand side; always above
                                 16 basis vectors): three passes over the
                                 basis per step                             */
#define R1S_ORTHO_CGS2 2      /* second pass on every step                 */

typedef struct {
  int iters;            /* Arnoldi steps (summed over inner solves)         */
  int cycles;           /* restart cycles                                   */
  int outer;            /* refinement steps (mixed mode)                    */
  int converged;        /* 1 if |b - J x| <= rtol |b|                       */
  double rel_residual;  /* true float64 relative residual at exit           */
} r1s_gmres_stats;

/* ---------------------------------------------------------------- API --- */

/* Message of the last failed call on this thread ("" if none). */
const char* r1s_last_error(void);

/* Device bytes of the packed matrix for an nx x ny mesh with L levels and
 * the block structure `layout` (NULL: one pair per block, band 1, no
 * coupling).  flags: R1S_KEEP_F32 adds float32 copies.  Errors: R1S_ERR_ARG
 * for nx, ny, L < 1, r_diag < 1, r_off < 0, band < 1, arrow not 0/1/2,
 * arrow = 2 with L < 2, or a NULL `bytes`; R1S_ERR_UNSUPPORTED for
 * L + 3 > R1S_MAX_M, r_diag > 9, r_off > 6 or band > R1S_MAX_BAND. */
int r1s_mat_size(int nx, int ny, int L, const r1s_layout* layout, int flags,
                 size_t* bytes);

/* Pack the structured arrays (see the layout above) into `mem` and create a
 * handle.  Section 5.1: the index structure is fixed by the mesh adjacency
 * and the block size by m; here it is implicit in (nx, ny, L).
 * Errors: R1S_ERR_ARG (dims, NULL or misaligned pointer, mem_bytes too
 * small), R1S_ERR_HIP. */
int r1s_mat_init(int nx, int ny, int L, const r1s_layout* layout, int flags,
                 const r1s_inputs* in, void* mem, size_t mem_bytes,
                 void* stream, r1s_mat* out);

/* New values, same structure (the next Newton iterate).  Preconditioners
 * and BSR copies made from A must be set up again. */
int r1s_mat_update(r1s_mat A, const r1s_inputs* in, void* stream);

int r1s_mat_destroy(r1s_mat A);

/* General 2-D mesh (section 5.1: the block structure of a BSR / BR1-BSR
 * matrix).  block_indptr [n_cells + 1] and block_indices [nnzb] are host
 * int32 arrays: the block columns of every block row, in any order, the
 * diagonal block exactly once; the structure must be symmetric (block (c, j)
 * exists iff (j, c) does, as for the faces of a finite-volume mesh) and a
 * row holds at most R1S_MAX_NBR off-diagonal blocks.  The library copies what
 * it needs; the arrays may be freed after the call.  Every other call
 * (matvec, residual, preconditioners, BSR copy, GMRES) takes the returned
 * handle like a structured one.  Errors: R1S_ERR_ARG for a malformed or
 * unsymmetric structure (the message names the row or block),
 * R1S_ERR_UNSUPPORTED for more than R1S_MAX_NBR neighbours or arrow = 2
 * (the atom coupling is built for the structured mesh), as for
 * r1s_mat_size / r1s_mat_init otherwise. */
int r1s_mat_size_graph(int n_cells, int L, const r1s_layout* layout,
                       const int* block_indptr, const int* block_indices,
                       int flags, size_t* bytes);
int r1s_mat_init_graph(int n_cells, int L, const r1s_layout* layout,
                       const int* block_indptr, const int* block_indices,
                       int flags, const r1s_graph_inputs* in, void* mem,
                       size_t mem_bytes, void* stream, r1s_mat* out);
/* New values for a general-mesh matrix (same structure). */
int r1s_mat_update_graph(r1s_mat A, const r1s_graph_inputs* in, void* stream);

/* General pattern of the diagonal block (section 4, Temporal Source
 * Jacobian: the nonzeros of S_{c,C} follow from the kinetic processes kept,
 * e.g. a Delta-v band, the DRa columns of the atom density and T, the flow
 * coupling, and are the same in every cell).  pattern_indptr [m + 1] and
 * pattern_indices [nnz] (host int32, CSR over the m = L + 3 unknowns of a
 * cell; each row lists its diagonal once, columns in any order) describe
 * S_{c,C} of every cell on the structured nx x ny mesh; its values come in
 * r1s_pattern_inputs.  layout gives r_diag and r_off; its band must be 1
 * and arrow 0 (the pattern replaces both).  The library copies what it
 * needs; the arrays may be freed after the call.
 *
 * The host analyses the pattern once: for the products it stores S_{c,C}
 * as its diagonal, ELL rows (at most 16 entries per row and per column)
 * and at most 8 dense rows / columns, choosing the split that stores the
 * fewest rows; for the block-Jacobi it orders the unknowns by minimum degree
 * and finds the fill of LU without pivoting, which every cell's numeric
 * factorisation (r1s_prec_setup) then follows, one lane per cell.  Every
 * other call (matvec, residual, preconditioner, BSR copy, GMRES) takes the
 * handle like a structured one.  Errors: R1S_ERR_ARG for a malformed
 * pattern (the message names the row) or band / arrow not 1 / 0,
 * R1S_ERR_UNSUPPORTED for a pattern that does not fit those limits, as for
 * r1s_mat_size / r1s_mat_init otherwise. */
int r1s_mat_size_pattern(int nx, int ny, int L, const r1s_layout* layout,
                         const int* pattern_indptr, const int* pattern_indices, int flags,
                         size_t* bytes);
int r1s_mat_init_pattern(int nx, int ny, int L, const r1s_layout* layout,
                         const int* pattern_indptr, const int* pattern_indices, int flags,
                         const r1s_pattern_inputs* in, void* mem, size_t mem_bytes,
                         void* stream, r1s_mat* out);
/* New values for a general-pattern matrix (same pattern). */
int r1s_mat_update_pattern(r1s_mat A, const r1s_pattern_inputs* in, void* stream);

/* Stored-value counts of the structured and dense-block representations
 * (section 3, Jacobian Complexity: N_A = sum m^2 (N_e + 1)). */
int r1s_mat_storage(r1s_mat A, r1s_storage* out);

/* y = J x (trans = 0) or y = J^T x (trans = 1) for nrhs vectors, section 5.2:
 * the sparse part plus, for every block, u times the coefficient v . x_col.
 * precision R1S_F32 needs R1S_KEEP_F32.  Asynchronous. */
int r1s_matvec(r1s_mat A, int precision, int trans, int nrhs, const double* x,
               double* y, void* stream);

/* r = b - J x in float64 (the residual of the refinement loop). */
int r1s_residual(r1s_mat A, int nrhs, const double* b, const double* x,
                 double* r, void* stream);

/* Device bytes for the SMW block-Jacobi factors of A (flags: R1S_KEEP_F32,
 * R1S_WITH_TRANS). */
int r1s_prec_size(r1s_mat A, int flags, size_t* bytes);

/* Section 6: block-Jacobi with D_c = A0_c + U_c V_c^T (eq. R1_Block_Jacobian;
 * the r_diag columns of U_c, V_c are the pairs of the diagonal block).
 * Factors the sparse diagonal block A0_c by LU without pivoting: the level
 * band (Thomas algorithm for band 1, banded LU otherwise), the flow corner
 * by its 3 x 3 inverse or, with level/flow coupling, by the inverse of its
 * 3 x 3 Schur complement; solves A0_c W_c = U_c (SMW-1), forms the
 * r_diag x r_diag capacitance C_c = I + V_c^T W_c (SMW-2) and inverts it
 * (Gauss-Jordan, partial pivoting).  With arrow = 2, A0_c leaves out the
 * atom's column c and row r, which join U_c, V_c as two more terms
 * (c, e_a) and (e_a, r): the capacitance is (r_diag + 2) square.  Synchronises; returns R1S_ERR_SINGULAR
 * naming the first cell with a zero pivot of A0_c or of C_c
 * (|pivot| <= 1e-12 (1 + |V_c| |W_c|), Frobenius norms). */
int r1s_prec_setup(r1s_mat A, int flags, void* mem, size_t mem_bytes,
                   void* stream, r1s_prec* out);

/* z = M r (trans = 0) or M^T r: per cell x0 = A0^{-1} r_c, then
 * z_c = x0 - W_c C_c^{-1} (V_c^T x0) (section 6, SMW steps, sign corrected;
 * the transpose uses A0^{-T} V_c, U_c and C_c^{-T}).
 * Also applies a BSR dense-LU preconditioner (r1s_bsr_prec_setup; trans = 0,
 * precision R1S_F64 only).  Asynchronous. */
int r1s_prec_apply(r1s_prec M, int precision, int trans, int nrhs,
                   const double* r, double* z, void* stream);

/* y = J x and z = M y in one call: the operator M J of the left-preconditioned
 * system (section 6, eq. left_precond_system), with J x kept.  M must be an
 * SMW preconditioner set up on A (R1S_ERR_ARG for another layout,
 * R1S_ERR_UNSUPPORTED for a BSR dense-LU one).  For one right-hand side on
 * the structured mesh with m <= 64, a tridiagonal level band without
 * level/flow coupling, and either one pair per block or float32 values, a
 * single kernel forms y_c and goes on to the local SMW solve of z_c in the
 * same wavefront (y is written, never read back); otherwise the call is
 * r1s_matvec followed by r1s_prec_apply.  The single
 * kernel gives the same y as r1s_matvec and z equal to r1s_prec_apply's up to
 * rounding (a few units in the last place).  precision R1S_F32 uses the float32
 * matrix values and the float32 factors (R1S_KEEP_F32 on both).  x, y, z:
 * device [nrhs][n] float64, caller-owned, pairwise distinct.  Asynchronous. */
int r1s_matvec_prec(r1s_mat A, r1s_prec M, int precision, int nrhs,
                    const double* x, double* y, double* z, void* stream);

int r1s_prec_destroy(r1s_prec M);

/* Dense-block BSR copy of A: every existing block D = S_{c,d} + sum u v^T stored
 * as a dense m x m block (section 5.1, BSR format; column-major inside a
 * block), plus block_indptr / block_indices (int32). */
int r1s_bsr_size(r1s_mat A, size_t* bytes);
int r1s_bsr_init(r1s_mat A, void* mem, size_t mem_bytes, void* stream,
                 r1s_bsr* out);
/* y = J x through the dense blocks.  Asynchronous. */
int r1s_bsr_matvec(r1s_bsr B, int nrhs, const double* x, double* y,
                   void* stream);
/* Classical block-Jacobi (section 6): LU with partial pivoting of every
 * diagonal dense block.  Synchronises; R1S_ERR_SINGULAR on a zero pivot. */
int r1s_bsr_prec_size(r1s_bsr B, size_t* bytes);
int r1s_bsr_prec_setup(r1s_bsr B, void* mem, size_t mem_bytes, void* stream,
                       r1s_prec* out);
int r1s_bsr_destroy(r1s_bsr B);

/* Workspace bytes for r1s_gmres with these options and nrhs. */
int r1s_gmres_work_size(r1s_mat A, const r1s_gmres_opts* opts, int nrhs,
                        size_t* bytes);

/* Restarted right-preconditioned GMRES (section 6): solves (J M) y = b and
 * returns x = M y, for nrhs independent right-hand sides advanced together.
 * Classical Gram-Schmidt with a second pass chosen by opts->ortho
 * (R1S_ORTHO_*), float64.  Mixed mode
 * wraps float32-operator inner solves in float64 iterative refinement: the
 * float64 residual b - J x before each inner solve (b itself from x = 0)
 * and after the last; an inner solve ends when its least-squares residual
 * estimate meets inner_rtol.
 * `B` is used when opts->op == R1S_OP_BSR (may be NULL otherwise).
 * On R1S_ERR_NOCONV, x holds the last iterate and stats are filled (one
 * r1s_gmres_stats per right-hand side, stats may be NULL).  Returns when the
 * solve's work on `stream` is complete and x is final: after synchronising
 * the stream, or after seeing its last kernel raise a ready flag in pinned
 * memory (that kernel's last write). */
int r1s_gmres(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts,
              int nrhs, const double* b, double* x, void* work,
              size_t work_bytes, r1s_gmres_stats* stats, void* stream);

/* r1s_gmres for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * solve (same options, same kernels, the same iterates and result as
 * r1s_gmres), with its workspace taken from a fixed array of
 * R1S_NOALLOC_MAX_BYTES bytes that the library holds on every GPU it runs on
 * until the process ends, instead of a caller-owned work buffer; and the
 * Arnoldi coefficients of each step staged in that array and copied to the
 * host, instead of through pinned host memory (one host wait per Arnoldi
 * step).  Allocates no device or pinned host memory (host-side bookkeeping
 * uses the C++ heap).  The caller still passes b and x (device [nrhs][N][m]
 * float64).  r1s_gmres_noalloc_size reports the bytes a solve needs; a solve
 * needing more than R1S_NOALLOC_MAX_BYTES fails with R1S_ERR_ARG before any
 * device work (use r1s_gmres).  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other threads, other streams) race and must
 * be serialised by the caller.  The array's contents are left over from the
 * last call; the solve needs none of them.  Errors and stats as r1s_gmres. */
#define R1S_NOALLOC_MAX_BYTES (64ull << 20)
int r1s_gmres_noalloc_size(r1s_mat A, const r1s_gmres_opts* opts, int nrhs,
                           size_t* bytes);
int r1s_gmres_noalloc(r1s_mat A, r1s_bsr B, r1s_prec M, const r1s_gmres_opts* opts,
                      int nrhs, const double* b, double* x, r1s_gmres_stats* stats,
                      void* stream);

/* Gradients of Loss with  J x_r = b_r  given lambda_r = J^{-T} dLoss/dx_r:
 * dLoss/dS = -sum_r lambda_r x_r^T on the stored pattern,
 * dLoss/du_{c,d,p} = -sum_r lambda_r[c] (v_{c,d,p} . x_r[nb]),
 * dLoss/dv_{c,d,p} = -sum_r x_r[nb] (u_{c,d,p} . lambda_r[c]); zero in the
 * slots of blocks that do not exist.  nrhs <= 64.  Asynchronous. */
int r1s_grad(r1s_mat A, int nrhs, const double* lambda, const double* x,
             const r1s_grads* out, void* stream);

/* The same gradients for a general-mesh matrix, in its input layout (zero
 * for no block: every listed block exists). */
int r1s_grad_graph(r1s_mat A, int nrhs, const double* lambda, const double* x,
                   const r1s_graph_grads* out, void* stream);

/* The same gradients for a general-pattern matrix: dLoss/ds_cc[c][e] =
 * -sum_r lambda_r[c][i] x_r[c][j] for entry e = (i, j) of the pattern. */
int r1s_grad_pattern(r1s_mat A, int nrhs, const double* lambda, const double* x,
                     const r1s_pattern_grads* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* R1S_H */
