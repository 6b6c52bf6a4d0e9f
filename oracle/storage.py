"""Stored-value counts of the two Jacobian representations.

Standard (BSR) representation, section 3: N_A = sum over elements of
m^2 (N_{kappa,e} + 1), where N_{kappa,e} is the element's number of interior
edges.  On a non-periodic nx x ny mesh the number of stored blocks is
B = 5N - 2nx - 2ny, so N_A = B m^2.

Block r1-sparse representation, sections 4-5: the fully sparse part stores,
per cell, the diagonal block pattern (m diagonal entries, 2(L-1) level-band
entries and 6 flow-corner entries: 3m - 2 in total since L = m - 3) and one
diagonal of m entries for each of the B - N neighbour blocks; the rank-one
part stores 2m values (u and v) per block and per pair.
"""


def n_blocks(nx: int, ny: int) -> int:
    """Count the stored blocks by walking the mesh (diagonal + interior edges)."""
    B = 0
    for iy in range(ny):
        for ix in range(nx):
            B += 1 + (iy > 0) + (ix > 0) + (ix < nx - 1) + (iy < ny - 1)
    return B


def bsr_values(nx: int, ny: int, m: int) -> int:
    return n_blocks(nx, ny) * m * m


def structured_values(nx: int, ny: int, m: int, r_diag: int = 1, r_off: int = 1,
                      band: int = 1, arrow: int = 0) -> int:
    """r_diag pairs on every diagonal block, r_off on every neighbour block;
    the diagonal block's level band has half-width `band` (2 (L - j) entries
    on the j-th diagonals), `arrow` adds 6 L level/flow couplings and
    arrow = 2 the atom's column and row over the molecule levels, of which
    the band already holds the 2 min(band, L - 1) positions next to the
    atom: 2 (L - 1 - band) more entries."""
    N = nx * ny
    B = n_blocks(nx, ny)
    L = m - 3
    diag_block = m + sum(2 * max(L - j, 0) for j in range(1, band + 1)) + 6
    if arrow:
        diag_block += 6 * L
    if arrow == 2:
        diag_block += 2 * max(L - 1 - band, 0)
    return N * diag_block + (B - N) * m + (N * r_diag + (B - N) * r_off) * 2 * m


def explicit_pattern_values(nx: int, ny: int, m: int, nnz: int, r_diag: int = 1,
                            r_off: int = 1) -> int:
    """Stored values with a general pattern of nnz entries (diagonal
    included) in every diagonal block: N nnz, plus the neighbour diagonals
    and the pairs as for the structured layouts."""
    N = nx * ny
    B = n_blocks(nx, ny)
    return N * nnz + (B - N) * m + 2 * m * (N * r_diag + (B - N) * r_off)
