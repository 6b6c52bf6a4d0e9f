"""Pins of the oracle's storage formats against the paper's worked examples
(section 5.1) and of its block rank-one product against dense algebra
(section 5.2)."""
import numpy as np
import scipy.sparse as sp

from conftest import load_golden
from oracle import formats


def test_csr_worked_example():
    g = load_golden("paper_csr_4x4.json")
    data, indices, indptr = formats.dense_to_csr(g["matrix"])
    assert data.tolist() == g["data"]
    assert indices.tolist() == g["indices"]
    assert indptr.tolist() == g["indptr"]
    A = np.array(g["matrix"], dtype=float)
    x = np.array([1.0, -2.0, 0.5, 3.0])
    assert np.array_equal(formats.csr_matvec(data, indices, indptr, x), A @ x)
    # scipy's CSR reading of the printed arrays is the same matrix
    M = sp.csr_array((g["data"], g["indices"], g["indptr"]), shape=(4, 4)).toarray()
    assert np.array_equal(M, A)


def test_r1_sparse_worked_example():
    g = load_golden("paper_r1_sparse.json")
    U = np.array(g["U"], dtype=float)
    Vt = np.array(g["Vt"], dtype=float)
    cols, rows = formats.r1_sparse(U, Vt.T)
    assert cols.tolist() == g["r1_columns"]
    assert rows.tolist() == g["r1_rows"]
    A = np.array(load_golden("paper_csr_4x4.json")["matrix"], dtype=float)
    x = np.array([0.25, -1.0, 2.0, 4.0])
    y = formats.r1_sparse_matvec(formats.dense_to_csr(A), cols, rows, x)
    assert np.allclose(y, (A + U @ Vt) @ x, rtol=0, atol=1e-12)


def test_bsr_worked_example():
    g = load_golden("paper_bsr_8x8.json")
    idx, ptr, data = formats.dense_to_bsr(g["matrix"], g["block_size"])
    assert idx.tolist() == g["block_indices"]
    assert ptr.tolist() == g["block_indptr"]
    assert data.tolist() == g["data"]
    M = sp.bsr_array((np.array(g["data"], dtype=float), g["block_indices"],
                      g["block_indptr"]), shape=(8, 8)).toarray()
    assert np.array_equal(M, np.array(g["matrix"], dtype=float))


def _br1_example(rng, pair_counts):
    g = load_golden("paper_br1_bsr.json")
    bs = g["block_size"]
    blocks = []
    for (I, J, _), k in zip(g["blocks"], pair_counts):
        blocks.append((I, J, [(rng.standard_normal(bs), rng.standard_normal(bs))
                              for _ in range(k)]))
    return g, blocks


def test_br1_bsr_worked_example_indices():
    rng = np.random.default_rng(3)
    g = load_golden("paper_br1_bsr.json")
    _, blocks = _br1_example(rng, [b[2] for b in g["blocks"]])
    br1 = formats.br1_bsr(blocks, 4)
    assert br1["block_indices"].tolist() == g["block_indices"]
    assert br1["block_indptr"].tolist() == g["block_indptr"]
    assert br1["pair_indptr"].tolist() == g["pair_indptr"]
    assert br1["column_pair_indptr"].tolist() == g["column_pair_indptr"]
    assert br1["column_data"].shape == (16, 2)


def _dense_of_pairs(blocks, nrows, bs):
    A = np.zeros((nrows * bs, nrows * bs))
    for I, J, pairs in blocks:
        for u, v in pairs:
            A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] += np.outer(u, v)
    return A


def test_br1_matvec_matches_dense_and_coeff_order():
    rng = np.random.default_rng(5)
    g = load_golden("paper_br1_bsr.json")
    for counts in ([b[2] for b in g["blocks"]], [1] * 8):
        _, blocks = _br1_example(rng, counts)
        br1 = formats.br1_bsr(blocks, 4)
        x = rng.standard_normal(8)
        y, coeffs = formats.br1_matvec(br1, x, 2, 2)
        A = _dense_of_pairs(blocks, 4, 2)
        assert np.allclose(y, A @ x, rtol=0, atol=1e-13)
        # section 5.2: column_coeffs holds v . x_J for every pair, in pair order
        expect = [float(np.dot(v, x[J * 2:(J + 1) * 2]))
                  for (_, J, pairs) in blocks for (_, v) in pairs]
        assert np.allclose(coeffs, expect, rtol=0, atol=1e-14)


def test_br1_matvec_accumulates_into_output():
    # the product adds into a pre-filled output (the CSR part's product)
    rng = np.random.default_rng(7)
    _, blocks = _br1_example(rng, [1] * 8)
    br1 = formats.br1_bsr(blocks, 4)
    x = rng.standard_normal(8)
    y0 = rng.standard_normal(8)
    y, _ = formats.br1_matvec(br1, x, 2, 2, y=y0.copy())
    assert np.allclose(y, y0 + _dense_of_pairs(blocks, 4, 2) @ x, rtol=0, atol=1e-13)
