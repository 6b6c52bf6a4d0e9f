"""Seeded synthetic inputs for the r1-sparse block Jacobian.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no matvec, no factorisation, no solve).  Both the HIP
library and the CPU oracle consume exactly the arrays produced here.

Problem family (the first-order finite-volume Jacobian of section 3 with the
block structure of section 4, "Overall Structure"): a structured nx x ny mesh,
5-point block stencil, block size m = L + 3 (L level densities, two momenta,
energy).  Every existing block (c, d) is  S_{c,d} + sum_p u_p v_p^T  over its
rank-one pairs (the block-wise rank-one representation of section 4).

Array layout (all float64, C-contiguous; N = nx*ny, cell c = iy*nx + ix):

  s_diag [N][m]      diagonal of S_cc
  s_sub  [N][L-1]    S_cc[k+1][k], level band (k = 0..L-2)
  s_sup  [N][L-1]    S_cc[k][k+1], level band
  s_flow [N][6]      flow-corner off-diagonals (rows/cols L..L+2) in the order
                     (0,1) (0,2) (1,0) (1,2) (2,0) (2,1)
  s_nbr  [N][4][m]   diagonals of the neighbour blocks S_{c,d}, d in S,W,E,N
  u, v   [N][P][m]   rank-one pairs grouped by block in the order S, W, C, E, N:
                     r_off pairs for each neighbour block and r_diag for the
                     diagonal block, P = r_diag + 4 r_off (P = 5 for one pair
                     per block)

Optional, for a wider sparse diagonal block (band > 1 and/or arrow):
  s_band     [N][2(band-1)][L]  further level diagonals: row j-2 holds
                                S_cc[k][k-j] and row band-1+j-2 holds
                                S_cc[k][k+j] at index k, j = 2..band
                                (entries outside the block are zero)
  s_lev_flow [N][3][L]          S_cc[k][L+i] at [c][i][k]: level rows coupled
                                to the flow unknowns (temperature dependence)
  s_flow_lev [N][3][L]          S_cc[L+i][k] at [c][i][k]: flow rows coupled
                                to the levels
  With arrow = 2 the last level a = L-1 is the atom density (DRa processes,
  section 4, "Temporal Source Jacobian") and both arrays are [N][4][L]:
  slot 3 holds the atom column S_cc[k][a] (s_lev_flow) and the atom row
  S_cc[a][k] (s_flow_lev) at index k < a; index a of slot 3 is unused (zero)
  and the level-band entries that reach the atom are drawn as zero.

Directions: 0 = S (iy-1), 1 = W (ix-1), 2 = C, 3 = E (ix+1), 4 = N (iy+1).
The paper's structure (section 4, "Overall Structure") has r_diag = 9 (one
source term and two per face) and r_off = 2 (two trace-flux terms); the
synthetic workloads default to one pair per block.
The mesh is not periodic: a boundary cell simply has no block towards the
missing neighbour, and the slots for such blocks are zero.

Value distributions (one fixed draw order from numpy's PCG64):
  s_diag = inv_dt + 10*|N(0,1)|, s_sub, s_sup, s_flow ~ N(0,1),
  s_nbr ~ U(-1,0), u, v ~ N(0, 0.1^2), then (only when requested) s_band ~
  N(0,1), s_lev_flow ~ N(0, 0.1^2), s_flow_lev ~ N(0,1)/L (row sums of the
  flow rows stay O(1) at any L), for arrow = 2 then the atom column
  ~ N(0, 0.1^2) and the atom row ~ N(0,1)/L.  Right-hand sides from seed+1, loss
  weights from seed+2, both N(0,1).  inv_dt = 20 makes S strictly row
  diagonally dominant with overwhelming probability; inv_dt = 1 is a stress
  case that forces GMRES restarts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict

import numpy as np

DIR_S, DIR_W, DIR_C, DIR_E, DIR_N = 0, 1, 2, 3, 4
# s_nbr slot j holds direction NBR_DIRS[j]
NBR_DIRS = (DIR_S, DIR_W, DIR_E, DIR_N)

FIELDS = ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v")
# arrays of the wider diagonal-block pattern (present when band > 1 or arrow)
PATTERN_FIELDS = ("s_band", "s_lev_flow", "s_flow_lev")


@dataclass(frozen=True)
class Workload:
    """A named problem size: mesh, levels, and solver settings."""
    name: str
    nx: int
    ny: int
    L: int
    restart: int = 50
    rtol: float = 1e-10
    nrhs: int = 1
    inv_dt: float = 20.0
    seed: int = 0

    @property
    def m(self) -> int:
        return self.L + 3

    @property
    def N(self) -> int:
        return self.nx * self.ny


# The five workloads of the benchmark plan: the small CPU-checkable case, the
# 256x128 L=61 single-GPU case, the 512x256 level sweep, the mixed-precision
# case and the batched adjoint case.
WORKLOADS: Dict[str, Workload] = {
    "small_16x16_L8": Workload("small_16x16_L8", 16, 16, 8, restart=30),
    "mesh256x128_L61": Workload("mesh256x128_L61", 256, 128, 61, restart=50),
    "mesh512x256_L32": Workload("mesh512x256_L32", 512, 256, 32),
    "mesh512x256_L61": Workload("mesh512x256_L61", 512, 256, 61),
    "mesh512x256_L120": Workload("mesh512x256_L120", 512, 256, 120),
    "mesh512x256_L200": Workload("mesh512x256_L200", 512, 256, 200),
    "adjoint256x128_L61_b8": Workload("adjoint256x128_L61_b8", 256, 128, 61,
                                      nrhs=8),
}
# The paper's rank structure: 9 pairs on diagonal blocks, 2 on the others.
PAPER_RANKS = (9, 2)


def block_exists(nx: int, ny: int) -> np.ndarray:
    """[N][5] bool: does cell c have a block in direction d (non-periodic)."""
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    ex = np.ones((nx * ny, 5), dtype=bool)
    ex[:, DIR_S] = iy > 0
    ex[:, DIR_W] = ix > 0
    ex[:, DIR_E] = ix < nx - 1
    ex[:, DIR_N] = iy < ny - 1
    return ex


def pair_slots(r_diag: int = 1, r_off: int = 1):
    """(first slot, count) of the pairs of each block direction S, W, C, E, N."""
    counts = (r_off, r_off, r_diag, r_off, r_off)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return [(int(a), int(b)) for a, b in zip(starts, counts)]


def _check_arrow(L: int, arrow: int) -> None:
    if arrow not in (0, 1, 2):
        raise ValueError("arrow must be 0, 1 or 2")
    if arrow == 2 and L < 2:
        raise ValueError("arrow = 2 needs L >= 2 (the atom plus a molecule level)")


def _draw_arrow(p, rng, N: int, L: int, band: int, arrow: int) -> None:
    """Level/flow coupling arrays (zero without arrow); arrow = 2 draws the
    atom slot after the three flow slots and clears what the atom replaces."""
    if not arrow:
        p["s_lev_flow"] = np.zeros((N, 3, L))
        p["s_flow_lev"] = np.zeros((N, 3, L))
        return
    p["s_lev_flow"] = 0.1 * rng.standard_normal((N, 3, L))
    p["s_flow_lev"] = rng.standard_normal((N, 3, L)) / L
    if arrow == 2:
        a = L - 1
        col = 0.1 * rng.standard_normal((N, 1, L))
        row = rng.standard_normal((N, 1, L)) / L
        col[:, 0, a] = 0.0
        row[:, 0, a] = 0.0
        p["s_lev_flow"] = np.concatenate([p["s_lev_flow"], col], axis=1)
        p["s_flow_lev"] = np.concatenate([p["s_flow_lev"], row], axis=1)
        # the atom is not a vibrational level: no band entries reach it
        if L >= 2:
            p["s_sub"][:, a - 1] = 0.0
            p["s_sup"][:, a - 1] = 0.0
        nb = band - 1
        for j in range(2, band + 1):
            if a - j >= 0:
                p["s_band"][:, j - 2, a] = 0.0        # S[a][a-j]
                p["s_band"][:, nb + j - 2, a - j] = 0.0  # S[a-j][a]


def make_problem(nx: int, ny: int, L: int, seed: int = 0, inv_dt: float = 20.0,
                 r_diag: int = 1, r_off: int = 1, band: int = 1,
                 arrow: int = 0) -> Dict[str, np.ndarray]:
    """Draw the structured values of one Jacobian (float64 arrays).  The
    returned dict also holds "ranks" = [r_diag, r_off] and, for a wider
    diagonal block, "pattern" = [band, arrow] with the PATTERN_FIELDS."""
    if nx < 1 or ny < 1 or L < 1:
        raise ValueError("nx, ny, L must be >= 1")
    if r_diag < 1 or r_off < 0:
        raise ValueError("need r_diag >= 1 and r_off >= 0")
    if band < 1:
        raise ValueError("need band >= 1")
    _check_arrow(L, arrow)
    N, m = nx * ny, L + 3
    P = r_diag + 4 * r_off
    rng = np.random.default_rng(seed)
    p = {}
    p["s_diag"] = inv_dt + 10.0 * np.abs(rng.standard_normal((N, m)))
    p["s_sub"] = rng.standard_normal((N, L - 1))
    p["s_sup"] = rng.standard_normal((N, L - 1))
    p["s_flow"] = rng.standard_normal((N, 6))
    p["s_nbr"] = rng.uniform(-1.0, 0.0, size=(N, 4, m))
    p["u"] = 0.1 * rng.standard_normal((N, P, m))
    p["v"] = 0.1 * rng.standard_normal((N, P, m))
    ex = block_exists(nx, ny)
    for j, d in enumerate(NBR_DIRS):
        p["s_nbr"][~ex[:, d], j, :] = 0.0
    for d, (a, cnt) in enumerate(pair_slots(r_diag, r_off)):
        p["u"][~ex[:, d], a:a + cnt, :] = 0.0
        p["v"][~ex[:, d], a:a + cnt, :] = 0.0
    wide = band > 1 or arrow
    if wide:
        nb = band - 1
        p["s_band"] = rng.standard_normal((N, 2 * nb, L))
        k = np.arange(L)
        for j in range(2, band + 1):
            p["s_band"][:, j - 2, k < j] = 0.0             # S[k][k-j] needs k >= j
            p["s_band"][:, nb + j - 2, k + j > L - 1] = 0.0  # S[k][k+j] needs k+j < L
        _draw_arrow(p, rng, N, L, band, arrow)
    for k in FIELDS + (PATTERN_FIELDS if wide else ()):
        p[k] = np.ascontiguousarray(p[k], dtype=np.float64)
    p["ranks"] = np.array([r_diag, r_off])
    if wide:
        p["pattern"] = np.array([band, int(arrow)])
    return p


def make_rhs(nx: int, ny: int, L: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Right-hand sides b ~ N(0,1), shape [nrhs][N][m], from seed+1."""
    rng = np.random.default_rng(seed + 1)
    return rng.standard_normal((nrhs, nx * ny, L + 3))


def make_loss_weights(nx: int, ny: int, L: int, nrhs: int = 1,
                      seed: int = 0) -> np.ndarray:
    """Loss weights w ~ N(0,1), shape [nrhs][N][m], from seed+2."""
    rng = np.random.default_rng(seed + 2)
    return rng.standard_normal((nrhs, nx * ny, L + 3))


def make_vector(nx: int, ny: int, L: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """A generic N(0,1) test vector [nrhs][N][m] from its own stream."""
    rng = np.random.default_rng(1_000_003 + seed)
    return rng.standard_normal((nrhs, nx * ny, L + 3))


# -------------------------------------------------- explicit S_cc pattern --
# A general sparsity pattern of the diagonal block, shared by every cell
# (section 4, "Temporal Source Jacobian": the pattern follows from the
# kinetic processes kept, e.g. a Delta-v band, DRa columns, flow coupling):
# pat_indptr [m+1], pat_indices [nnz] (int32, CSR; each row lists its
# diagonal once, columns in any order) and s_cc [N][nnz], the values in the
# pattern's entry order.  The neighbour blocks and the pairs are as for the
# structured layouts (s_nbr, u, v, "ranks").
PATTERN_PROBLEM_FIELDS = ("s_cc", "s_nbr", "u", "v")


def layout_pattern(L: int, band: int = 1, arrow: int = 0):
    """The CSR pattern of S_cc of a structured layout (band, arrow): the
    diagonal, the level band, the flow corner, the level/flow coupling and,
    with arrow = 2, the atom's column and row; rows in ascending columns."""
    m = L + 3
    rows = [set([i]) for i in range(m)]
    for k in range(L):
        for j in range(1, band + 1):
            if k - j >= 0:
                rows[k].add(k - j)
            if k + j < L:
                rows[k].add(k + j)
    for i in range(3):
        for j in range(3):
            rows[L + i].add(L + j)
    if arrow:
        for k in range(L):
            for i in range(3):
                rows[k].add(L + i)
                rows[L + i].add(k)
    if arrow == 2:
        a = L - 1
        for k in range(a):
            rows[k].add(a)
            rows[a].add(k)
    indptr = np.zeros(m + 1, dtype=np.int32)
    indices = []
    for i in range(m):
        cols = sorted(rows[i])
        indices += cols
        indptr[i + 1] = indptr[i] + len(cols)
    return indptr, np.array(indices, dtype=np.int32)


def random_pattern(m: int, per_row: int = 3, dense_rows=(), dense_cols=(), seed: int = 0,
                   shuffle: bool = True):
    """A random pattern: the diagonal, per_row random off-diagonal columns
    in every row, full rows `dense_rows` and full columns `dense_cols`; each
    row's entries in random order when `shuffle`."""
    rng = np.random.default_rng(seed)
    rows = [set([i]) for i in range(m)]
    for i in range(m):
        others = [j for j in range(m) if j != i]
        for j in rng.choice(others, size=min(per_row, m - 1), replace=False):
            rows[i].add(int(j))
    for i in dense_rows:
        rows[i] |= set(range(m))
    for j in dense_cols:
        for i in range(m):
            rows[i].add(j)
    indptr = np.zeros(m + 1, dtype=np.int32)
    indices = []
    for i in range(m):
        cols = sorted(rows[i])
        if shuffle:
            cols = list(rng.permutation(cols))
        indices += [int(c) for c in cols]
        indptr[i + 1] = indptr[i] + len(cols)
    return indptr, np.array(indices, dtype=np.int32)


def make_pattern_problem(nx: int, ny: int, L: int, indptr, indices, seed: int = 0,
                         inv_dt: float = 20.0, r_diag: int = 1,
                         r_off: int = 1) -> Dict[str, np.ndarray]:
    """Values of a Jacobian whose diagonal blocks share the pattern (indptr,
    indices): diagonal entries inv_dt + 10 |N(0,1)|, the off-diagonal ones of
    a row with k of them N(0,1) min(1, 4 / k) (row sums of |S| stay about 3,
    so the block stays dominant), then s_nbr ~ U(-1, 0), u, v ~ N(0, 0.1^2)
    as in make_problem."""
    indptr = np.asarray(indptr, dtype=np.int32)
    indices = np.asarray(indices, dtype=np.int32)
    N, m = nx * ny, L + 3
    if len(indptr) != m + 1:
        raise ValueError("pattern must have m + 1 = L + 4 row pointers")
    P = r_diag + 4 * r_off
    rng = np.random.default_rng(seed)
    nnz = int(indptr[-1])
    row = np.repeat(np.arange(m), np.diff(indptr))
    diag = indices == row
    off_count = np.diff(indptr) - 1
    scale = np.minimum(1.0, 4.0 / np.maximum(off_count, 1))[row]
    z = rng.standard_normal((N, nnz))
    p = {"pat_indptr": indptr.copy(), "pat_indices": indices.copy()}
    p["s_cc"] = np.where(diag[None, :], inv_dt + 10.0 * np.abs(z), z * scale[None, :])
    p["s_nbr"] = rng.uniform(-1.0, 0.0, size=(N, 4, m))
    p["u"] = 0.1 * rng.standard_normal((N, P, m))
    p["v"] = 0.1 * rng.standard_normal((N, P, m))
    ex = block_exists(nx, ny)
    for j, d in enumerate(NBR_DIRS):
        p["s_nbr"][~ex[:, d], j, :] = 0.0
    for d, (a, cnt) in enumerate(pair_slots(r_diag, r_off)):
        p["u"][~ex[:, d], a:a + cnt, :] = 0.0
        p["v"][~ex[:, d], a:a + cnt, :] = 0.0
    for k in PATTERN_PROBLEM_FIELDS:
        p[k] = np.ascontiguousarray(p[k], dtype=np.float64)
    p["ranks"] = np.array([r_diag, r_off])
    return p


def workload_problem(w: Workload) -> Dict[str, np.ndarray]:
    return make_problem(w.nx, w.ny, w.L, seed=w.seed, inv_dt=w.inv_dt)


# ------------------------------------------------------------- general mesh --
# A general 2-D mesh is given by its block structure in the index arrays of
# the BR1-BSR format (section 5.1): block_indptr [N+1] and block_indices
# [nnzb] (int32), the block columns of every block row, the diagonal block
# included once.  The adjacency is structurally symmetric (a face joins two
# cells).  Off-diagonal blocks are numbered in the order of block_indices,
# skipping each row's diagonal entry.
GRAPH_FIELDS = ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u_diag", "v_diag", "u_off",
                "v_off")


def structured_graph(nx: int, ny: int):
    """Index arrays of the structured nx x ny mesh (blocks S, W, C, E, N)."""
    indptr, indices = [0], []
    for c in range(nx * ny):
        iy, ix = divmod(c, nx)
        cols = []
        if iy > 0:
            cols.append(c - nx)
        if ix > 0:
            cols.append(c - 1)
        cols.append(c)
        if ix < nx - 1:
            cols.append(c + 1)
        if iy < ny - 1:
            cols.append(c + nx)
        indices += cols
        indptr.append(len(indices))
    return np.array(indptr, dtype=np.int32), np.array(indices, dtype=np.int32)


def delaunay_graph(n_points: int, seed: int = 0, shuffle: bool = True):
    """Cell adjacency of a Delaunay triangulation of random points in the unit
    square: every triangle is a cell, neighbours share an edge (at most 3).
    Rows list the diagonal first, then the neighbours in ascending order.
    With `shuffle`, cells are renumbered at random (no locality)."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    tri = Delaunay(rng.random((n_points, 2)))
    nbrs = tri.neighbors  # [n_tri][3], -1 on the hull
    n = nbrs.shape[0]
    perm = rng.permutation(n) if shuffle else np.arange(n)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)          # old -> new
    indptr, indices = [0], []
    for new in range(n):
        old = perm[new]
        cols = sorted(int(inv[t]) for t in nbrs[old] if t >= 0)
        indices += [new] + cols
        indptr.append(len(indices))
    return np.array(indptr, dtype=np.int32), np.array(indices, dtype=np.int32)


def graph_off_blocks(indptr, indices):
    """(row, column) of every off-diagonal block in input order."""
    rows, cols = [], []
    for c in range(len(indptr) - 1):
        for b in range(indptr[c], indptr[c + 1]):
            if indices[b] != c:
                rows.append(c)
                cols.append(int(indices[b]))
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def make_graph_problem(indptr, indices, L: int, seed: int = 0, inv_dt: float = 20.0,
                       r_diag: int = 1, r_off: int = 1, band: int = 1,
                       arrow: int = 0) -> Dict[str, np.ndarray]:
    """Structured values on a general mesh, same distributions as
    make_problem: per cell the diagonal block (s_diag, s_sub, s_sup, s_flow,
    optional s_band / s_lev_flow / s_flow_lev, r_diag pairs u_diag, v_diag
    [N][r_diag][m]); per off-diagonal block its diagonal s_nbr [n_off][m]
    and r_off pairs u_off, v_off [n_off][r_off][m]."""
    _check_arrow(L, arrow)
    N, m = len(indptr) - 1, L + 3
    n_off = len(indices) - N
    rng = np.random.default_rng(seed)
    p = {"graph_indptr": np.asarray(indptr, dtype=np.int32),
         "graph_indices": np.asarray(indices, dtype=np.int32)}
    p["s_diag"] = inv_dt + 10.0 * np.abs(rng.standard_normal((N, m)))
    p["s_sub"] = rng.standard_normal((N, L - 1))
    p["s_sup"] = rng.standard_normal((N, L - 1))
    p["s_flow"] = rng.standard_normal((N, 6))
    p["s_nbr"] = rng.uniform(-1.0, 0.0, size=(n_off, m))
    p["u_diag"] = 0.1 * rng.standard_normal((N, r_diag, m))
    p["v_diag"] = 0.1 * rng.standard_normal((N, r_diag, m))
    p["u_off"] = 0.1 * rng.standard_normal((n_off, r_off, m))
    p["v_off"] = 0.1 * rng.standard_normal((n_off, r_off, m))
    wide = band > 1 or arrow
    if wide:
        nb = band - 1
        p["s_band"] = rng.standard_normal((N, 2 * nb, L))
        k = np.arange(L)
        for j in range(2, band + 1):
            p["s_band"][:, j - 2, k < j] = 0.0
            p["s_band"][:, nb + j - 2, k + j > L - 1] = 0.0
        _draw_arrow(p, rng, N, L, band, arrow)
        p["pattern"] = np.array([band, int(arrow)])
    for k in GRAPH_FIELDS + (PATTERN_FIELDS if wide else ()):
        p[k] = np.ascontiguousarray(p[k], dtype=np.float64)
    p["ranks"] = np.array([r_diag, r_off])
    return p


def graph_from_structured(p: Dict[str, np.ndarray], nx: int, ny: int) -> Dict[str, np.ndarray]:
    """The same Jacobian as a structured problem, in the general-mesh layout
    (blocks of missing neighbours dropped; a re-layout, no arithmetic)."""
    r_diag, r_off = (int(v) for v in p.get("ranks", (1, 1)))
    slots = pair_slots(r_diag, r_off)
    indptr, indices = structured_graph(nx, ny)
    q = {"graph_indptr": indptr, "graph_indices": indices, "ranks": np.array([r_diag, r_off])}
    for k in ("s_diag", "s_sub", "s_sup", "s_flow") + tuple(k for k in PATTERN_FIELDS if k in p):
        q[k] = p[k].copy()
    if "pattern" in p:
        q["pattern"] = p["pattern"].copy()
    a, cnt = slots[DIR_C]
    q["u_diag"] = p["u"][:, a:a + cnt].copy()
    q["v_diag"] = p["v"][:, a:a + cnt].copy()
    nbr, uo, vo = [], [], []
    for c in range(nx * ny):
        iy, ix = divmod(c, nx)
        for d, ok in ((DIR_S, iy > 0), (DIR_W, ix > 0), (DIR_E, ix < nx - 1), (DIR_N, iy < ny - 1)):
            if ok:
                nbr.append(p["s_nbr"][c, NBR_DIRS.index(d)])
                a, cnt = slots[d]
                uo.append(p["u"][c, a:a + cnt])
                vo.append(p["v"][c, a:a + cnt])
    m = p["s_diag"].shape[1]
    n_off = len(nbr)
    q["s_nbr"] = np.array(nbr).reshape(n_off, m)
    q["u_off"] = np.array(uo).reshape(n_off, r_off, m)
    q["v_off"] = np.array(vo).reshape(n_off, r_off, m)
    return q
