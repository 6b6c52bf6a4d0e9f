"""The C ABI without a GPU: the library loads, exports every declared
symbol, and rejects bad arguments on the host before any device work."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT
from paper_2403_09198_amd import _lib as L

HEADER = os.path.join(ROOT, "include", "r1s.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(r1s_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_bound_calls():
    assert _declared() == sorted(L.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _lay(r_diag, r_off, band=1, arrow=0):
    return C.byref(L.Layout(r_diag=r_diag, r_off=r_off, band=band, arrow=arrow))


def _rc(code_call):
    rc = code_call
    msg = L.lib().r1s_last_error().decode()
    return rc, msg


def test_size_validation():
    lib = L.lib()
    b = C.c_size_t()
    assert lib.r1s_mat_size(0, 4, 4, _lay(1, 1), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert "must be >= 1" in lib.r1s_last_error().decode()
    assert lib.r1s_mat_size(4, 4, 0, _lay(1, 1), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 254, _lay(1, 1), 0, C.byref(b)) == L.R1S_ERR_UNSUPPORTED
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1), 0, None) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1), 0x10, C.byref(b)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 253, _lay(1, 1), 1, C.byref(b)) == L.R1S_OK
    # packed rows are padded to 8 values: 17 rows of 256 doubles + floats
    assert b.value >= 16 * 17 * 256 * 12


def test_rank_validation():
    lib = L.lib()
    b = C.c_size_t()
    assert lib.r1s_mat_size(4, 4, 4, _lay(0, 1), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert "r_diag" in lib.r1s_last_error().decode()
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, -1), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 4, _lay(10, 2), 0, C.byref(b)) == L.R1S_ERR_UNSUPPORTED
    assert lib.r1s_mat_size(4, 4, 4, _lay(9, 7), 0, C.byref(b)) == L.R1S_ERR_UNSUPPORTED
    for rd, ro in ((9, 2), (1, 0), (2, 0), (3, 1), (8, 6)):
        assert lib.r1s_mat_size(4, 4, 4, _lay(rd, ro), 0, C.byref(b)) == L.R1S_OK
        # one record of 7 + 2 (rd + 4 ro) rows of m = 7 doubles per cell
        # (rows shorter than 64 values are not padded)
        assert b.value >= 16 * (7 + 2 * (rd + 4 * ro)) * 7 * 8


def test_layout_validation_and_sizes():
    lib = L.lib()
    b, a = C.c_size_t(), C.c_size_t()
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1, 0), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1, 1, 3), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1, 1, -1), 0, C.byref(b)) == L.R1S_ERR_ARG
    # the atom coupling needs the atom and at least one molecule level
    assert lib.r1s_mat_size(4, 4, 1, _lay(1, 1, 1, 2), 0, C.byref(b)) == L.R1S_ERR_ARG
    assert "L >= 2" in lib.r1s_last_error().decode()
    assert lib.r1s_mat_size(4, 4, 4, _lay(1, 1, L.R1S_MAX_BAND + 1), 0, C.byref(b)) == \
        L.R1S_ERR_UNSUPPORTED
    # NULL layout = one pair per block, band 1, no coupling
    assert lib.r1s_mat_size(8, 4, 61, None, 0, C.byref(a)) == L.R1S_OK
    assert lib.r1s_mat_size(8, 4, 61, _lay(1, 1), 0, C.byref(b)) == L.R1S_OK
    assert a.value == b.value
    # band 4 with coupling: 2 (4 - 1) + 6 more rows of 64 doubles per cell
    assert lib.r1s_mat_size(8, 4, 61, _lay(1, 1, 4, 1), 0, C.byref(b)) == L.R1S_OK
    assert b.value - a.value == 32 * 12 * 64 * 8
    # the atom's column and row: two more rows
    c = C.c_size_t()
    assert lib.r1s_mat_size(8, 4, 61, _lay(1, 1, 4, 2), 0, C.byref(c)) == L.R1S_OK
    assert c.value - b.value == 32 * 2 * 64 * 8


def test_init_requires_pattern_arrays():
    lib = L.lib()
    ins = L.Inputs()
    h = C.c_void_p()
    fake = C.c_void_p(1 << 20)
    for k in ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v"):
        setattr(ins, k, 1 << 21)
    assert lib.r1s_mat_init(4, 4, 4, _lay(1, 1, 3), 0, C.byref(ins), fake, 1 << 30, None,
                            C.byref(h)) == L.R1S_ERR_ARG
    assert "s_band" in lib.r1s_last_error().decode()
    ins.s_band = 1 << 21
    assert lib.r1s_mat_init(4, 4, 4, _lay(1, 1, 3, 1), 0, C.byref(ins), fake, 1 << 30, None,
                            C.byref(h)) == L.R1S_ERR_ARG
    assert "s_lev_flow" in lib.r1s_last_error().decode()


def test_size_grows_with_pairs():
    lib = L.lib()
    a, b = C.c_size_t(), C.c_size_t()
    lib.r1s_mat_size(64, 32, 61, _lay(1, 1), 0, C.byref(a))
    lib.r1s_mat_size(64, 32, 61, _lay(9, 2), 0, C.byref(b))
    mp = 64
    assert b.value - a.value == 64 * 32 * 2 * (17 - 5) * mp * 8


def test_size_is_linear_in_cells():
    lib = L.lib()
    a, b = C.c_size_t(), C.c_size_t()
    lib.r1s_mat_size(64, 32, 61, _lay(1, 1), 0, C.byref(a))
    lib.r1s_mat_size(128, 32, 61, _lay(1, 1), 0, C.byref(b))
    assert abs(b.value - 2 * a.value) <= 512


def test_init_rejects_bad_arguments_before_device_work():
    lib = L.lib()
    ins = L.Inputs()
    h = C.c_void_p()
    fake = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert lib.r1s_mat_init(4, 4, 4, None, 0, None, fake, 1 << 30, None, C.byref(h)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_init(4, 4, 4, None, 0, C.byref(ins), fake, 1 << 30, None, C.byref(h)) == L.R1S_ERR_ARG
    assert "is NULL" in lib.r1s_last_error().decode()
    for k in ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v"):
        setattr(ins, k, 1 << 21)
    ins.u = (1 << 21) + 4  # misaligned
    assert lib.r1s_mat_init(4, 4, 4, None, 0, C.byref(ins), fake, 1 << 30, None, C.byref(h)) == L.R1S_ERR_ARG
    assert "aligned" in lib.r1s_last_error().decode()
    ins.u = 1 << 21
    assert lib.r1s_mat_init(4, 4, 4, None, 0, C.byref(ins), fake, 16, None, C.byref(h)) == L.R1S_ERR_ARG
    assert "mem_bytes" in lib.r1s_last_error().decode()
    assert lib.r1s_mat_init(4, 4, 4, None, 0, C.byref(ins), C.c_void_p((1 << 20) + 8), 1 << 30, None,
                            C.byref(h)) == L.R1S_ERR_ARG
    assert lib.r1s_mat_init(4, 4, 4, None, 0, C.byref(ins), fake, 1 << 30, None, None) == L.R1S_ERR_ARG


def test_null_handles_rejected():
    lib = L.lib()
    fake = C.c_void_p(1 << 20)
    assert lib.r1s_matvec(None, 0, 0, 1, fake, fake, None) == L.R1S_ERR_ARG
    assert lib.r1s_prec_apply(None, 0, 0, 1, fake, fake, None) == L.R1S_ERR_ARG
    assert lib.r1s_matvec_prec(None, fake, 0, 1, fake, fake, fake, None) == L.R1S_ERR_ARG
    assert "matrix handle" in lib.r1s_last_error().decode()
    assert lib.r1s_matvec_prec(fake, None, 0, 1, fake, fake, fake, None) == L.R1S_ERR_ARG
    assert "preconditioner handle" in lib.r1s_last_error().decode()
    assert lib.r1s_bsr_matvec(None, 1, fake, fake, None) == L.R1S_ERR_ARG
    assert lib.r1s_mat_storage(None, None) == L.R1S_ERR_ARG
    assert lib.r1s_grad(None, 1, fake, fake, None, None) == L.R1S_ERR_ARG
    opts = L.GmresOpts(restart=10, max_cycles=5, rtol=1e-8)
    assert lib.r1s_gmres(None, None, None, C.byref(opts), 1, fake, fake, fake, 1 << 30, None,
                         None) == L.R1S_ERR_ARG
    assert lib.r1s_mat_destroy(None) == L.R1S_OK


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        L.lib()


def _graph_size(indptr, indices, lay=None):
    lib = L.lib()
    b = C.c_size_t()
    ip = (C.c_int * len(indptr))(*indptr)
    ix = (C.c_int * len(indices))(*indices)
    rc = lib.r1s_mat_size_graph(len(indptr) - 1, 4, lay, ip, ix, 0, C.byref(b))
    return rc, lib.r1s_last_error().decode(), b.value


def test_general_mesh_structure_is_validated():
    # two cells joined by a face: fine
    assert _graph_size([0, 2, 4], [0, 1, 1, 0])[0] == L.R1S_OK
    # missing diagonal, diagonal twice, out of range, duplicate, unsymmetric
    assert _graph_size([0, 1, 3], [1, 1, 0])[0] == L.R1S_ERR_ARG
    rc, msg, _ = _graph_size([0, 2, 3], [0, 0, 1])
    assert rc == L.R1S_ERR_ARG and "twice" in msg
    assert _graph_size([0, 2, 4], [0, 5, 1, 0])[0] == L.R1S_ERR_ARG
    rc, msg, _ = _graph_size([0, 2, 3], [0, 1, 1])
    assert rc == L.R1S_ERR_ARG and "transposed partner" in msg
    assert _graph_size([1, 2, 4], [0, 1, 1, 0])[0] == L.R1S_ERR_ARG
    # a star: cell 0 has 9 neighbours (more than 8)
    n = 10
    ix = list(range(n))       # row 0: itself and cells 1..9
    ip = [0, n]
    for c in range(1, n):
        ix += [0, c]          # row c: cell 0 and itself
        ip.append(ip[-1] + 2)
    assert _graph_size(ip, ix)[0] == L.R1S_ERR_UNSUPPORTED


def test_general_mesh_rejects_the_atom_coupling():
    rc, msg, _ = _graph_size([0, 2, 4], [0, 1, 1, 0], _lay(1, 1, 1, 2))
    assert rc == L.R1S_ERR_UNSUPPORTED and "structured mesh" in msg
    assert _graph_size([0, 2, 4], [0, 1, 1, 0], _lay(1, 1, 1, 1))[0] == L.R1S_OK


def test_general_mesh_size_matches_structured_record():
    # a 4 x 3 structured mesh as a graph: the same record plus int32 tables
    from paper_2403_09198_amd import gen
    ip, ix = gen.structured_graph(4, 3)
    rc, _, gb = _graph_size(list(ip), list(ix), _lay(1, 1))
    assert rc == L.R1S_OK
    b = C.c_size_t()
    assert L.lib().r1s_mat_size(4, 3, 4, _lay(1, 1), 0, C.byref(b)) == L.R1S_OK
    assert gb > b.value and gb - b.value <= 3 * 256 + 4 * (2 * 12 * 4 + 12)


def test_noalloc_gmres_rejects_null_handles():
    lib = L.lib()
    b = C.c_size_t()
    opts = L.GmresOpts(restart=10, max_cycles=5, rtol=1e-8)
    assert lib.r1s_gmres_noalloc_size(None, C.byref(opts), 1, C.byref(b)) == L.R1S_ERR_ARG
    st = (L.GmresStats * 1)()
    assert lib.r1s_gmres_noalloc(None, None, None, C.byref(opts), 1, None, None, st,
                                 None) == L.R1S_ERR_ARG
    assert "NULL" in lib.r1s_last_error().decode()
