"""Structured-mesh adjacency for the first-order finite-volume stencil.

Section 3 ("Jacobian Complexity"): the block row of element kappa holds the
diagonal block plus one block per interior edge of kappa.  On a structured
nx x ny quadrilateral mesh without periodicity an element has up to four
interior edges (section 4, "Overall Structure").

Cell numbering: c = iy*nx + ix.  Direction numbering: 0 = S (iy-1),
1 = W (ix-1), 2 = C (the cell itself), 3 = E (ix+1), 4 = N (iy+1); for a given
cell these are in ascending order of the neighbour's cell number.
"""
import numpy as np

S, W, C, E, N = 0, 1, 2, 3, 4
# slot of each off-diagonal direction in the [N][4][m] neighbour-diagonal array
NBR_SLOT = {S: 0, W: 1, E: 2, N: 3}


def neighbour(nx: int, ny: int, c: int, d: int) -> int:
    """Cell number of the neighbour of c in direction d, or -1 if none."""
    iy, ix = divmod(c, nx)
    if d == S:
        return c - nx if iy > 0 else -1
    if d == W:
        return c - 1 if ix > 0 else -1
    if d == C:
        return c
    if d == E:
        return c + 1 if ix < nx - 1 else -1
    if d == N:
        return c + nx if iy < ny - 1 else -1
    raise ValueError(d)


def neighbour_table(nx: int, ny: int) -> np.ndarray:
    """[N][5] int array of neighbour cell numbers (-1 where no block)."""
    tab = np.full((nx * ny, 5), -1, dtype=np.int64)
    for c in range(nx * ny):
        for d in range(5):
            tab[c, d] = neighbour(nx, ny, c, d)
    return tab


def neighbour_table_row(nx: int, ny: int, c: int):
    """Neighbours of c in the order S, W, C, E, N (-1 where none)."""
    return [neighbour(nx, ny, c, d) for d in range(5)]


def pair_range(p, d: int):
    """Slots (start, count) of the rank-one pairs of the block in direction d.

    Section 4 ("Overall Structure"): a diagonal block carries the source
    term's pair and two per face, an off-diagonal block the two trace-flux
    pairs.  The arrays u, v hold the pairs of a cell's blocks one after the
    other in the order S, W, C, E, N: r_off pairs for each neighbour block,
    r_diag for the diagonal block (p["ranks"] = [r_diag, r_off], default one
    pair each)."""
    r_diag, r_off = (int(v) for v in p.get("ranks", (1, 1)))
    counts = [r_off, r_off, r_diag, r_off, r_off]
    return sum(counts[:d]), counts[d]


def pattern(p):
    """(band, arrow) of the diagonal sparse block: level diagonals up to
    |k - k'| <= band, and whether level rows and flow rows are coupled (the
    temperature dependence of the level sources, section 4, "Temporal Source
    Jacobian"; arrow = 2 adds the atom density, the last level, coupled to
    every level by the DRa processes).  Default (1, 0): tridiagonal band, no
    coupling."""
    if "pat_indptr" in p:
        return 0, 0  # explicit pattern: no structured band (see explicit_pattern)
    if "pattern" not in p:
        return 1, 0
    band, arrow = (int(v) for v in p["pattern"])
    return band, arrow


def explicit_pattern(p):
    """(indptr, indices) of a general pattern of S_cc shared by every cell
    (values s_cc [N][nnz] in entry order), or None for the structured
    layouts."""
    if "pat_indptr" not in p:
        return None
    return p["pat_indptr"], p["pat_indices"]


def opposite(d: int) -> int:
    """The direction pointing back: the neighbour's block towards c."""
    return {S: N, W: E, C: C, E: W, N: S}[d]
