// Host check of the general-pattern plan (csrc/pattern.hip), run by
// tests/test_pattern_plan.py without a GPU.  Reads patterns from stdin:
//   m nnz  indptr[m+1]  indices[nnz]   (repeated; m = 0 ends)
// and for each one builds the plan, then checks that every table index is
// in range, that the record layout (diagonal, ELL rows, dense rows and
// columns) and the transposed ELL hold each entry exactly once, and that
// LU without pivoting and the four triangular solves driven by the plan's
// tables reproduce a dense Gaussian elimination on a random dominant matrix
// with that pattern.  Prints "ok <m> <nnz> <ne> <net> <ns> <nnzF>" per
// pattern or "FAIL <reason>" / "ERR <code> <message>".
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "pattern.hpp"

using namespace r1s;

static int fails = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      printf("FAIL ");                    \
      printf(__VA_ARGS__);                \
      printf("\n");                       \
      ++fails;                            \
      return;                             \
    }                                     \
  } while (0)

static void check_plan(int m, const std::vector<int>& ip, const std::vector<int>& ix) {
  PatternPlan P;
  char msg[256] = "";
  const int rc = build_pattern_plan(m, ip.data(), ix.data(), &P, msg, sizeof msg);
  if (rc != 0) {
    printf("ERR %d %s\n", rc, msg);
    return;
  }
  const int nnz = ip[m], mp = P.mp;
  const int fb = F_BAND, fa = fb + P.ne, fu = fa + 2 * P.ns;
  CHECK(P.nnz == nnz && P.ne <= PAT_ELL_MAX && P.net <= PAT_ELL_MAX && P.ns <= PAT_SLOTS_MAX,
        "limits");
  // every entry at its own record element, inside the pattern rows
  std::vector<int> seen((size_t)fu * mp, -1);
  for (int e = 0; e < nnz; ++e) {
    const int o = P.eoff[e], f = o / mp, k = o % mp;
    CHECK(o >= 0 && f < fu && k < m && (f == F_DIAG || f >= fb), "entry %d offset %d", e, o);
    CHECK(seen[o] < 0, "entries %d and %d share element %d", seen[o], e, o);
    seen[o] = e;
    const int i = P.erow[e], j = P.ecol[e];
    // what the matvec reads at that element: the entry's row and column
    int ri = -1, cj = -1;
    if (f == F_DIAG) {
      ri = cj = k;
    } else if (f < fa) {
      ri = k;
      cj = P.pcol[(size_t)(f - fb) * mp + k];
    } else if (f < fa + P.ns) {
      ri = k;
      cj = P.px[f - fa];
    } else {
      ri = P.px[f - fa - P.ns];
      cj = k;
    }
    CHECK(ri == i && cj == j, "entry %d (%d,%d) read as (%d,%d)", e, i, j, ri, cj);
    CHECK(P.pack[(size_t)(f == F_DIAG ? 0 : f - fb + 1) * mp + k] == e, "pack of entry %d", e);
    CHECK(P.dense[(size_t)i * m + j] == e, "dense table of entry %d", e);
  }
  int npack = 0;
  for (int v : P.pack) npack += v >= 0;
  CHECK(npack == nnz, "pack lists %d entries", npack);
  // the ELL columns of absent entries point at the lane itself (value zero)
  for (int s = 0; s < P.ne; ++s)
    for (int k = 0; k < m; ++k) {
      const int c = P.pcol[(size_t)s * mp + k];
      CHECK(c >= 0 && c < m, "pcol range");
      const int o = (fb + s) * mp + k;
      CHECK(seen[o] >= 0 || c == k, "empty ELL slot %d lane %d points at %d", s, k, c);
    }
  // transposed ELL: every ELL entry once, at its column's lane
  std::vector<int> tcount(nnz, 0);
  for (int t = 0; t < P.net; ++t)
    for (int k = 0; k < m; ++k) {
      const int o = P.ptpos[(size_t)t * mp + k], r = P.ptcol[(size_t)t * mp + k];
      CHECK(r >= 0 && r < m, "ptcol range");
      if (o < 0) continue;
      CHECK(o < fu * mp && seen[o] >= 0, "ptpos %d", o);
      const int e = seen[o];
      CHECK(P.ecol[e] == k && P.erow[e] == r, "transposed ELL entry %d", e);
      ++tcount[e];
    }
  for (int e = 0; e < nnz; ++e) {
    const int f = P.eoff[e] / mp;
    const bool ell = f >= fb && f < fa;
    CHECK(tcount[e] == (ell ? 1 : 0), "entry %d in the transposed ELL %d times", e, tcount[e]);
  }
  // the packed lane tables the kernels read decode to the same slots
  std::vector<int> c8, t16;
  pattern_lane_tables(P, c8, t16);
  for (int k = 0; k < m; ++k)
    for (int s = 0; s < PAT_ELL_MAX; ++s) {
      const unsigned cw = (unsigned)c8[(size_t)k * (PAT_ELL_MAX / 4) + s / 4];
      const int col = (int)((cw >> (8 * (s % 4))) & 0xffu);
      if (s < P.ne) CHECK(col == P.pcol[(size_t)s * mp + k], "packed column slot %d lane %d", s, k);
      const unsigned tw = (unsigned)t16[(size_t)k * (PAT_ELL_MAX / 2) + s / 2];
      const unsigned h = (tw >> (16 * (s % 2))) & 0xffffu;
      const int o = s < P.net ? P.ptpos[(size_t)s * mp + k] : -1;
      if (o < 0) {
        CHECK(h == 0xffffu, "packed transposed slot %d lane %d should be empty", s, k);
      } else {
        CHECK((int)((F_BAND + (h >> 8)) * mp + (h & 0xffu)) == o &&
                  (int)(h & 0xffu) == P.ptcol[(size_t)s * mp + k],
              "packed transposed slot %d lane %d", s, k);
      }
    }
  // LU tables
  const int nF = P.nnzF;
  std::vector<int> isperm(m, 0);
  for (int i = 0; i < m; ++i) {
    CHECK(P.perm[i] >= 0 && P.perm[i] < m && !isperm[P.perm[i]]++, "perm");
    CHECK(P.dpos[i] >= 0 && P.dpos[i] < nF, "dpos");
  }
  for (int p = 0; p < nF; ++p) {
    const int o = P.frec[p];
    CHECK(o == -1 || (o >= 0 && o < fu * mp && seen[o] >= 0), "frec %d", p);
  }
  auto rng_ok = [&](const std::vector<int>& ptr, const std::vector<int>& pos) {
    if ((int)ptr.size() != m + 1 || ptr[0] != 0 || ptr[m] != (int)pos.size()) return false;
    for (int v : pos)
      if (v < 0 || v >= nF) return false;
    return true;
  };
  CHECK(rng_ok(P.lrow_ptr, P.lrow_pos) && rng_ok(P.urow_ptr, P.urow_pos) &&
            rng_ok(P.lcol_ptr, P.lcol_pos) && rng_ok(P.ucol_ptr, P.ucol_pos),
        "LU table ranges");
  CHECK((int)P.lrow_pos.size() + (int)P.urow_pos.size() + m == nF, "L + U + diagonal = nnzF");

  // numeric check: random dominant values on the pattern
  std::mt19937_64 gen(12345 + m + nnz);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> rec((size_t)fu * mp, 0.0), A((size_t)m * m, 0.0);
  for (int e = 0; e < nnz; ++e) {
    const int i = P.erow[e], j = P.ecol[e];
    const double v = i == j ? 20.0 + 10.0 * fabs(nd(gen)) : nd(gen) / (1.0 + (ip[i + 1] - ip[i]) / 4.0);
    rec[P.eoff[e]] = v;
    A[(size_t)i * m + j] = v;
  }
  // the plan's LU (the arithmetic of the setup kernel, one cell)
  std::vector<double> F(nF);
  for (int p = 0; p < nF; ++p) F[p] = P.frec[p] >= 0 ? rec[P.frec[p]] : 0.0;
  for (int k = 0; k < m; ++k) {
    const double inv = 1.0 / F[P.dpos[k]];
    F[P.dpos[k]] = inv;
    for (int a = P.lcol_ptr[k]; a < P.lcol_ptr[k + 1]; ++a) {
      const double l = F[P.lcol_pos[a]] * inv;
      F[P.lcol_pos[a]] = l;
      const int i = P.lcol_row[a];
      for (int b = P.urow_ptr[k]; b < P.urow_ptr[k + 1]; ++b) {
        const int pij = P.posF[(size_t)i * m + P.urow_col[b]];
        CHECK(pij >= 0, "fill missing at (%d,%d)", i, P.urow_col[b]);
        F[pij] -= l * F[P.urow_pos[b]];
      }
    }
  }
  auto solve = [&](bool trans, std::vector<double>& v) {
    if (!trans) {
      for (int i = 0; i < m; ++i) {
        double y = v[P.perm[i]];
        for (int e = P.lrow_ptr[i]; e < P.lrow_ptr[i + 1]; ++e) y -= F[P.lrow_pos[e]] * v[P.lrow_oc[e]];
        v[P.perm[i]] = y;
      }
      for (int i = m - 1; i >= 0; --i) {
        double x = v[P.perm[i]];
        for (int e = P.urow_ptr[i]; e < P.urow_ptr[i + 1]; ++e) x -= F[P.urow_pos[e]] * v[P.urow_oc[e]];
        v[P.perm[i]] = x * F[P.dpos[i]];
      }
    } else {
      for (int i = 0; i < m; ++i) {
        double z = v[P.perm[i]];
        for (int e = P.ucol_ptr[i]; e < P.ucol_ptr[i + 1]; ++e) z -= F[P.ucol_pos[e]] * v[P.ucol_or[e]];
        v[P.perm[i]] = z * F[P.dpos[i]];
      }
      for (int i = m - 1; i >= 0; --i) {
        double x = v[P.perm[i]];
        for (int e = P.lcol_ptr[i]; e < P.lcol_ptr[i + 1]; ++e) x -= F[P.lcol_pos[e]] * v[P.lcol_or[e]];
        v[P.perm[i]] = x;
      }
    }
  };
  // the flat operation streams the apply kernel runs
  auto stream = [&](bool trans, std::vector<double>& v) -> bool {
    const std::vector<int>& ops = trans ? P.ops_t : P.ops_n;
    double acc = 0.0;
    for (size_t e = 0; e + 1 < ops.size(); e += 2) {
      const int pos = ops[e], kind = ops[e + 1] >> 16, idx = ops[e + 1] & 0xffff;
      if (idx < 0 || idx >= m || pos < -1 || pos >= nF) return false;
      if (kind == PAT_OP_UPD) {
        if (pos < 0) return false;
        acc -= F[pos] * v[idx];
      } else if (kind == PAT_OP_START) {
        acc = v[idx];
      } else if (kind == PAT_OP_END) {
        v[idx] = pos >= 0 ? acc * F[pos] : acc;
      } else {
        return false;
      }
    }
    return true;
  };
  for (int trans = 0; trans < 2; ++trans) {
    std::vector<double> b(m), x(m);
    for (int i = 0; i < m; ++i) b[i] = nd(gen);
    x = b;
    solve(trans, x);
    std::vector<double> xs = b;
    CHECK(stream(trans, xs), "stream (trans %d) out of range", trans);
    for (int i = 0; i < m; ++i) CHECK(xs[i] == x[i], "stream (trans %d) differs at %d", trans, i);
    // residual of A x = b (A^T x = b) against |A| |x| + |b|
    double worst = 0.0;
    for (int i = 0; i < m; ++i) {
      double r = b[i], sc = fabs(b[i]);
      for (int j = 0; j < m; ++j) {
        const double a = trans ? A[(size_t)j * m + i] : A[(size_t)i * m + j];
        r -= a * x[j];
        sc += fabs(a * x[j]);
      }
      worst = fmax(worst, fabs(r) / sc);
    }
    CHECK(worst < 1e-13, "solve (trans %d) residual %.3g", trans, worst);
  }
  printf("ok %d %d %d %d %d %d\n", m, nnz, P.ne, P.net, P.ns, nF);
}

int main() {
  int m, nnz;
  while (scanf("%d %d", &m, &nnz) == 2 && m > 0) {
    std::vector<int> ip(m + 1), ix(nnz);
    for (int& v : ip)
      if (scanf("%d", &v) != 1) return 2;
    for (int& v : ix)
      if (scanf("%d", &v) != 1) return 2;
    check_plan(m, ip, ix);
  }
  return fails ? 1 : 0;
}
