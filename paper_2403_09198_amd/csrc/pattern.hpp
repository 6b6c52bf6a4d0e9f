// Host analysis of a general sparsity pattern of the diagonal block S_cc,
// shared by every cell (section 4, "Temporal Source Jacobian": which entries
// of S_cc are nonzero follows from the kinetic processes kept and is the
// same in every cell).
//
// The matvec stores S_cc in the record as its diagonal, up to PAT_ELL_MAX
// "ELL" rows (entry s of row k at lane k, its column in a shared table) and
// up to PAT_SLOTS_MAX dense indices X (a row row, S[X][k] at lane k, and a
// column row, S[k][X] at lane k), the split chosen to store the fewest rows.
// The block-Jacobi factors S_cc by LU without pivoting after a symmetric
// minimum-degree ordering; the symbolic factorisation (fill) is done here
// once, and every cell's numeric factorisation and solves follow the same
// position tables.
#pragma once
#include <stddef.h>

#include <vector>

#include "r1s_device.hpp"

namespace r1s {

struct PatternPlan {
  int m = 0, mp = 0, nnz = 0;
  std::vector<int> erow, ecol;  // [nnz] row and column of each entry
  // matvec layout (record rows: F_DIAG, fb .. fb + ne - 1, fa .. fa + 2 ns - 1)
  int ne = 0, net = 0, ns = 0;
  int px[PAT_SLOTS_MAX] = {0};
  std::vector<int> eoff;          // [nnz] offset of each entry in a cell's record
  std::vector<int> pcol;          // [ne][mp] column of ELL entry s at lane k
  std::vector<int> ptpos, ptcol;  // [net][mp] transposed ELL: record offset, row
  std::vector<int> pack;          // [1 + ne + 2 ns][mp] entry feeding each record element, -1
  std::vector<int> dense;         // [m][m] entry at (i, j), -1
  // LU of P S_cc P^T, positions p of the filled pattern (row-major, new order)
  int nnzF = 0;
  std::vector<int> perm;          // new index -> original index
  std::vector<int> frec;          // [nnzF] record offset of the value, -1 for fill
  std::vector<int> dpos;          // [m]
  std::vector<int> posF;          // [m][m] position, -1 outside the filled pattern
  // strict lower L and strict upper U by rows and by columns: position, the
  // other index in the new order, and that index in the original order
  std::vector<int> lrow_ptr, lrow_pos, lrow_oc;
  std::vector<int> urow_ptr, urow_pos, urow_col, urow_oc;
  std::vector<int> lcol_ptr, lcol_pos, lcol_row, lcol_or;
  std::vector<int> ucol_ptr, ucol_pos, ucol_or;
  // The two solves as flat operation streams (forward then backward sweep),
  // 2 ints per operation: (factor position or -1, kind << 16 | index) with
  // kind PAT_OP_START (acc = v[index]), PAT_OP_UPD (acc -= F[pos] v[index])
  // or PAT_OP_END (v[index] = acc, times F[pos] when pos >= 0).  ops_n
  // solves A0 x = r, ops_t A0^T x = r.
  std::vector<int> ops_n, ops_t;
};

// Validates the CSR pattern (m + 1 row pointers from 0, columns in range,
// no column twice in a row, the diagonal in every row) and builds the plan.
// Returns R1S_OK or an r1s error code with a message in msg.
int build_pattern_plan(int m, const int* indptr, const int* indices, PatternPlan* out, char* msg,
                       size_t msg_len);

// The LU tables in one int array (the order of PatLU's members) and their
// offsets; `dev` is where the array will live, for the pointers.
void pattern_lu_tables(const PatternPlan& p, std::vector<int>& out, const int* dev, PatLU* lu);

// The ELL tables as the kernels read them, one lane's slots together: c8
// [mp][PAT_ELL_MAX / 4] (the column of slot s of lane k in byte s), t16 [mp]
// [PAT_ELL_MAX / 2] (transposed slot s of lane (column) k in halfword s:
// the entry's ELL slot << 8 | its row, 0xffff for none).
void pattern_lane_tables(const PatternPlan& p, std::vector<int>& c8, std::vector<int>& t16);

// The matvec tables in one int array and the Mesh pointers into `dev`.
void pattern_mat_tables(const PatternPlan& p, std::vector<int>& out, const int* dev, Mesh* g);

}  // namespace r1s
