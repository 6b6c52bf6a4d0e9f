// Host analysis of a general pattern of the diagonal block (see pattern.hpp).
#include "pattern.hpp"

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>

#include "r1s.h"

namespace r1s {

static int perr(char* msg, size_t len, int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  if (msg && len) vsnprintf(msg, len, fmt, ap);
  va_end(ap);
  return code;
}

namespace {

// A set of indices 0 .. m-1 as a bit array (m <= R1S_MAX_M).
struct Bits {
  uint64_t w[(R1S_MAX_M + 63) / 64] = {0};
  void set(int i) { w[i >> 6] |= 1ull << (i & 63); }
  bool has(int i) const { return (w[i >> 6] >> (i & 63)) & 1; }
};

// The split of the off-diagonal entries into dense-index rows / columns and
// ELL rows.  Greedy: while the ELL part is too wide (more than PAT_ELL_MAX
// entries in a row or a column), or while it lowers the stored rows (ELL
// width + 2 per dense index), move the fullest remaining row or column to a
// dense index; the row wins ties.  Fails with more than PAT_SLOTS_MAX dense
// indices.
struct Split {
  std::vector<char> drow, dcol;
  int w = 0, wt = 0, ns = 0;
};

struct Counts {
  int w, wt, ns, imax, jmax;
};

Counts count(int m, const std::vector<int>& er, const std::vector<int>& ec, const Split& sp) {
  std::vector<int> rc(m, 0), cc(m, 0);
  for (size_t e = 0; e < er.size(); ++e) {
    const int i = er[e], j = ec[e];
    if (i == j || sp.drow[i] || sp.dcol[j]) continue;
    ++rc[i];
    ++cc[j];
  }
  Counts c{0, 0, 0, 0, 0};
  for (int i = 0; i < m; ++i) {
    if (rc[i] > c.w) { c.w = rc[i]; c.imax = i; }
    if (cc[i] > c.wt) { c.wt = cc[i]; c.jmax = i; }
    c.ns += sp.drow[i] || sp.dcol[i];
  }
  return c;
}

bool split_pattern(int m, const std::vector<int>& er, const std::vector<int>& ec, Split* out) {
  Split sp;
  sp.drow.assign(m, 0);
  sp.dcol.assign(m, 0);
  for (;;) {
    const Counts c = count(m, er, ec, sp);
    if (c.ns > PAT_SLOTS_MAX) return false;
    const bool fits = c.w <= PAT_ELL_MAX && c.wt <= PAT_ELL_MAX;
    if (c.w == 0 && c.wt == 0) {  // nothing left in the ELL part
      sp.w = sp.wt = 0;
      sp.ns = c.ns;
      *out = sp;
      return true;
    }
    Split a = sp, b = sp;
    a.drow[c.imax] = 1;
    b.dcol[c.jmax] = 1;
    const Counts ca = count(m, er, ec, a), cb = count(m, er, ec, b);
    const int cost = c.w + 2 * c.ns, cost_a = ca.w + 2 * ca.ns, cost_b = cb.w + 2 * cb.ns;
    const bool take_row = c.w >= c.wt;  // the fuller of the two
    if (!fits) {
      sp = take_row ? a : b;
      continue;
    }
    const int best = std::min(cost_a, cost_b);
    if (best < cost && std::max(ca.ns, cb.ns) <= PAT_SLOTS_MAX) {
      const bool pick_a = cost_a < cost_b || (cost_a == cost_b && take_row);
      if ((pick_a ? ca.ns : cb.ns) <= PAT_SLOTS_MAX) {
        sp = pick_a ? a : b;
        continue;
      }
    }
    sp.w = c.w;
    sp.wt = c.wt;
    sp.ns = c.ns;
    *out = sp;
    return true;
  }
}

}  // namespace

int build_pattern_plan(int m, const int* indptr, const int* indices, PatternPlan* out, char* msg,
                       size_t msg_len) {
  if (m < 1 || m > R1S_MAX_M) return perr(msg, msg_len, R1S_ERR_ARG, "block size %d out of range", m);
  if (!indptr || !indices) return perr(msg, msg_len, R1S_ERR_ARG, "pattern_indptr or pattern_indices is NULL");
  if (indptr[0] != 0) return perr(msg, msg_len, R1S_ERR_ARG, "pattern_indptr[0] must be 0");
  PatternPlan& P = *out;
  P = PatternPlan();
  P.m = m;
  P.mp = pad_m(m);
  const int mp = P.mp;
  P.dense.assign((size_t)m * m, -1);
  for (int i = 0; i < m; ++i) {
    if (indptr[i + 1] < indptr[i])
      return perr(msg, msg_len, R1S_ERR_ARG, "pattern_indptr decreases at row %d", i);
    if (indptr[i + 1] - indptr[i] > m)
      return perr(msg, msg_len, R1S_ERR_ARG, "pattern row %d has more than m entries", i);
    bool diag = false;
    for (int e = indptr[i]; e < indptr[i + 1]; ++e) {
      const int j = indices[e];
      if (j < 0 || j >= m) return perr(msg, msg_len, R1S_ERR_ARG, "pattern column %d of row %d out of range", j, i);
      if (P.dense[(size_t)i * m + j] >= 0)
        return perr(msg, msg_len, R1S_ERR_ARG, "pattern row %d lists column %d twice", i, j);
      P.dense[(size_t)i * m + j] = e;
      P.erow.push_back(i);
      P.ecol.push_back(j);
      diag = diag || j == i;
    }
    if (!diag) return perr(msg, msg_len, R1S_ERR_ARG, "pattern row %d has no diagonal entry", i);
  }
  P.nnz = indptr[m];

  // --- matvec split
  Split best;
  if (!split_pattern(m, P.erow, P.ecol, &best))
    return perr(msg, msg_len, R1S_ERR_UNSUPPORTED,
                "pattern needs more than %d dense rows / columns to keep at most %d other "
                "entries per row and column", PAT_SLOTS_MAX, PAT_ELL_MAX);
  P.ne = best.w;
  P.net = best.wt;
  std::vector<int> slot(m, -1);
  for (int i = 0; i < m; ++i)
    if (best.drow[i] || best.dcol[i]) {
      slot[i] = P.ns;
      P.px[P.ns++] = i;
    }
  const int fb = F_BAND, fa = F_BAND + P.ne;
  P.eoff.assign(P.nnz, -1);
  P.pcol.assign((size_t)P.ne * mp, 0);
  for (int s = 0; s < P.ne; ++s)
    for (int k = 0; k < mp; ++k) P.pcol[(size_t)s * mp + k] = std::min(k, m - 1);
  std::vector<int> fill(m, 0);
  for (int e = 0; e < P.nnz; ++e) {
    const int i = P.erow[e], j = P.ecol[e];
    if (i == j) {
      P.eoff[e] = F_DIAG * mp + i;
    } else if (best.drow[i]) {
      P.eoff[e] = (fa + P.ns + slot[i]) * mp + j;
    } else if (best.dcol[j]) {
      P.eoff[e] = (fa + slot[j]) * mp + i;
    } else {
      const int s = fill[i]++;
      P.eoff[e] = (fb + s) * mp + i;
      P.pcol[(size_t)s * mp + i] = j;
    }
  }
  // transposed ELL: the ELL entries of column j
  P.ptpos.assign((size_t)P.net * mp, -1);
  P.ptcol.assign((size_t)P.net * mp, 0);
  for (int t = 0; t < P.net; ++t)
    for (int k = 0; k < mp; ++k) P.ptcol[(size_t)t * mp + k] = std::min(k, m - 1);
  std::vector<int> tfill(m, 0);
  for (int e = 0; e < P.nnz; ++e) {
    const int i = P.erow[e], j = P.ecol[e];
    const int f = P.eoff[e] / mp;
    if (f < fb || f >= fa) continue;
    const int t = tfill[j]++;
    P.ptpos[(size_t)t * mp + j] = P.eoff[e];
    P.ptcol[(size_t)t * mp + j] = i;
  }
  // pack gather: record rows F_DIAG, fb .., fa .. -> pack rows 0, 1 .., 1 + ne ..
  const int prows = 1 + P.ne + 2 * P.ns;
  P.pack.assign((size_t)prows * mp, -1);
  for (int e = 0; e < P.nnz; ++e) {
    const int f = P.eoff[e] / mp, k = P.eoff[e] % mp;
    const int r = f == F_DIAG ? 0 : f - fb + 1;
    P.pack[(size_t)r * mp + k] = e;
  }

  // --- ordering: minimum degree on the symmetrised pattern (ties: lowest index)
  std::vector<Bits> adj(m);
  for (int e = 0; e < P.nnz; ++e) {
    const int i = P.erow[e], j = P.ecol[e];
    if (i == j) continue;
    adj[i].set(j);
    adj[j].set(i);
  }
  std::vector<char> gone(m, 0);
  P.perm.clear();
  for (int step = 0; step < m; ++step) {
    int v = -1, dv = 0;
    for (int i = 0; i < m; ++i) {
      if (gone[i]) continue;
      int d = 0;
      for (int j = 0; j < m; ++j) d += !gone[j] && adj[i].has(j);
      if (v < 0 || d < dv) {
        v = i;
        dv = d;
      }
    }
    P.perm.push_back(v);
    gone[v] = 1;
    std::vector<int> nb;
    for (int j = 0; j < m; ++j)
      if (!gone[j] && adj[v].has(j)) nb.push_back(j);
    for (int a : nb)
      for (int b : nb)
        if (a != b) adj[a].set(b);
  }
  std::vector<int> inew(m);
  for (int i = 0; i < m; ++i) inew[P.perm[i]] = i;

  // --- symbolic LU of B = P S P^T (right-looking, fill by row unions)
  std::vector<Bits> B(m);
  for (int e = 0; e < P.nnz; ++e) B[inew[P.erow[e]]].set(inew[P.ecol[e]]);
  for (int k = 0; k < m; ++k)
    for (int i = k + 1; i < m; ++i) {
      if (!B[i].has(k)) continue;
      for (int j = k + 1; j < m; ++j)
        if (B[k].has(j)) B[i].set(j);
    }
  P.posF.assign((size_t)m * m, -1);
  P.nnzF = 0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      if (B[i].has(j)) P.posF[(size_t)i * m + j] = P.nnzF++;
  P.frec.assign(P.nnzF, -1);
  P.dpos.assign(m, -1);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const int p = P.posF[(size_t)i * m + j];
      if (p < 0) continue;
      const int e = P.dense[(size_t)P.perm[i] * m + P.perm[j]];
      P.frec[p] = e >= 0 ? P.eoff[e] : -1;
      if (i == j) P.dpos[i] = p;
    }
  auto csr = [&](bool lower, bool by_row, std::vector<int>& ptr, std::vector<int>& pos,
                 std::vector<int>* other_new, std::vector<int>* other_orig) {
    ptr.assign(m + 1, 0);
    pos.clear();
    if (other_new) other_new->clear();
    if (other_orig) other_orig->clear();
    for (int a = 0; a < m; ++a) {
      for (int b = 0; b < m; ++b) {
        const int i = by_row ? a : b, j = by_row ? b : a;  // entry (i, j)
        if (lower ? !(j < i) : !(j > i)) continue;
        const int p = P.posF[(size_t)i * m + j];
        if (p < 0) continue;
        pos.push_back(p);
        if (other_new) other_new->push_back(b);
        if (other_orig) other_orig->push_back(P.perm[b]);
      }
      ptr[a + 1] = (int)pos.size();
    }
  };
  csr(true, true, P.lrow_ptr, P.lrow_pos, nullptr, &P.lrow_oc);
  csr(false, true, P.urow_ptr, P.urow_pos, &P.urow_col, &P.urow_oc);
  csr(true, false, P.lcol_ptr, P.lcol_pos, &P.lcol_row, &P.lcol_or);
  csr(false, false, P.ucol_ptr, P.ucol_pos, nullptr, &P.ucol_or);

  // flat solve streams
  auto op = [](std::vector<int>& v, int pos, int kind, int idx) {
    v.push_back(pos);
    v.push_back(kind << 16 | idx);
  };
  auto sweep = [&](std::vector<int>& v, bool up, const std::vector<int>& ptr,
                   const std::vector<int>& pos, const std::vector<int>& other, bool scale) {
    for (int t = 0; t < m; ++t) {
      const int i = up ? t : m - 1 - t;
      op(v, -1, PAT_OP_START, P.perm[i]);
      for (int e = ptr[i]; e < ptr[i + 1]; ++e) op(v, pos[e], PAT_OP_UPD, other[e]);
      op(v, scale ? P.dpos[i] : -1, PAT_OP_END, P.perm[i]);
    }
  };
  P.ops_n.clear();
  sweep(P.ops_n, true, P.lrow_ptr, P.lrow_pos, P.lrow_oc, false);
  sweep(P.ops_n, false, P.urow_ptr, P.urow_pos, P.urow_oc, true);
  P.ops_t.clear();
  sweep(P.ops_t, true, P.ucol_ptr, P.ucol_pos, P.ucol_or, true);
  sweep(P.ops_t, false, P.lcol_ptr, P.lcol_pos, P.lcol_or, false);
  return R1S_OK;
}

void pattern_lu_tables(const PatternPlan& p, std::vector<int>& out, const int* dev, PatLU* lu) {
  out.clear();
  auto add = [&](const std::vector<int>& v) -> const int* {
    const size_t o = out.size();
    out.insert(out.end(), v.begin(), v.end());
    while (out.size() % 64) out.push_back(0);  // 256-byte aligned pieces
    return dev ? dev + o : nullptr;
  };
  lu->nnzF = p.nnzF;
  lu->nops_n = (int)p.ops_n.size() / 2;
  lu->nops_t = (int)p.ops_t.size() / 2;
  lu->ops_n = add(p.ops_n);
  lu->ops_t = add(p.ops_t);
  lu->perm = add(p.perm);
  lu->frec = add(p.frec);
  lu->dpos = add(p.dpos);
  lu->posF = add(p.posF);
  lu->lrow_ptr = add(p.lrow_ptr);
  lu->lrow_pos = add(p.lrow_pos);
  lu->lrow_oc = add(p.lrow_oc);
  lu->urow_ptr = add(p.urow_ptr);
  lu->urow_pos = add(p.urow_pos);
  lu->urow_col = add(p.urow_col);
  lu->urow_oc = add(p.urow_oc);
  lu->lcol_ptr = add(p.lcol_ptr);
  lu->lcol_pos = add(p.lcol_pos);
  lu->lcol_row = add(p.lcol_row);
  lu->lcol_or = add(p.lcol_or);
  lu->ucol_ptr = add(p.ucol_ptr);
  lu->ucol_pos = add(p.ucol_pos);
  lu->ucol_or = add(p.ucol_or);
}

void pattern_lane_tables(const PatternPlan& p, std::vector<int>& c8, std::vector<int>& t16) {
  const int mp = p.mp;
  c8.assign((size_t)mp * (PAT_ELL_MAX / 4), 0);
  t16.assign((size_t)mp * (PAT_ELL_MAX / 2), 0);
  for (int k = 0; k < mp; ++k) {
    for (int s = 0; s < PAT_ELL_MAX; ++s) {
      const unsigned col = s < p.ne ? (unsigned)p.pcol[(size_t)s * mp + k] : 0u;
      c8[(size_t)k * (PAT_ELL_MAX / 4) + s / 4] |= (int)((col & 0xffu) << (8 * (s % 4)));
      unsigned h = 0xffffu;
      if (s < p.net && p.ptpos[(size_t)s * mp + k] >= 0) {
        const int o = p.ptpos[(size_t)s * mp + k];
        h = (unsigned)((o / mp - F_BAND) << 8 | (o % mp));
      }
      t16[(size_t)k * (PAT_ELL_MAX / 2) + s / 2] |= (int)(h << (16 * (s % 2)));
    }
  }
}

void pattern_mat_tables(const PatternPlan& p, std::vector<int>& out, const int* dev, Mesh* g) {
  out.clear();
  auto add = [&](const std::vector<int>& v) -> const int* {
    const size_t o = out.size();
    out.insert(out.end(), v.begin(), v.end());
    while (out.size() % 64) out.push_back(0);
    return dev ? dev + o : nullptr;
  };
  std::vector<int> c8, t16;
  pattern_lane_tables(p, c8, t16);
  g->pcol = add(c8);
  g->ptpos = add(t16);
  g->ptcol = nullptr;
  g->ppack = add(p.pack);
  g->perow = add(p.erow);
  g->pecol = add(p.ecol);
  g->peoff = add(p.eoff);
  g->pdense = add(p.dense);
}

}  // namespace r1s
