"""Python binding of the r1s C ABI.

Functions named like the C calls (r1s_mat_size, r1s_matvec, ...) marshal
torch tensors into pointers and sizes and nothing else: every step runs in
the HIP kernels of libr1s.so.  torch supplies device memory and the stream.
The classes below (R1Matrix, SMWPreconditioner, BSRMatrix) keep the
caller-owned device buffers alive next to the handles.

Vectors are float64 CUDA tensors of shape [nrhs, N, m] or [N, m].
"""
import ctypes as C
from dataclasses import dataclass
from typing import Dict, List, Optional

import torch

from . import _lib as L
from ._lib import R1SError, check, lib

FIELDS = ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v")
# arrays of the wide diagonal-block pattern (band > 1 or level/flow coupling)
PATTERN_FIELDS = ("s_band", "s_lev_flow", "s_flow_lev")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _need_vec(t, name, n):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() % n != 0 or t.numel() == 0:
        raise ValueError(f"{name} has {t.numel()} elements, not a multiple of N*m = {n}")
    return t.numel() // n


def _buffer(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def layout(r_diag=1, r_off=1, band=1, arrow=0) -> "L.Layout":
    """arrow: 0 none, 1 (or True) level/flow coupling, 2 also the atom density
    coupled to every molecule level."""
    return L.Layout(r_diag=int(r_diag), r_off=int(r_off), band=int(band), arrow=int(arrow))


def _used_fields(lay):
    """The arrays a layout reads, in r1s_inputs order."""
    extra = (("s_band",) if lay.band > 1 else ()) + (
        ("s_lev_flow", "s_flow_lev") if lay.arrow else ())
    return FIELDS + extra


def _shapes(nx, ny, Lv, lay):
    N, m = nx * ny, Lv + 3
    P = lay.r_diag + 4 * lay.r_off
    return {"s_diag": (N, m), "s_sub": (N, Lv - 1), "s_sup": (N, Lv - 1), "s_flow": (N, 6),
            "s_nbr": (N, 4, m), "u": (N, P, m), "v": (N, P, m),
            "s_band": (N, 2 * (lay.band - 1), Lv), "s_lev_flow": (N, _slots(lay), Lv),
            "s_flow_lev": (N, _slots(lay), Lv)}


def _slots(lay):
    """Coupling slots of the level/flow arrays: the three flow unknowns, and
    the atom with arrow = 2."""
    return 4 if lay.arrow == 2 else 3


def _inputs(values: Dict[str, torch.Tensor], nx, ny, Lv, lay):
    shapes = _shapes(nx, ny, Lv, lay)
    ins = L.Inputs()
    for k in _used_fields(lay):
        t = values[k]
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
            raise TypeError(f"{k} must be a float64 CUDA tensor")
        if tuple(t.shape) != shapes[k] or not t.is_contiguous():
            raise ValueError(f"{k} must be contiguous with shape {shapes[k]}")
        setattr(ins, k, _ptr(t).value)
    return ins


# ----------------------------------------------------- C-named functions ---
def r1s_last_error() -> str:
    return lib().r1s_last_error().decode()


def r1s_mat_size(nx, ny, Lv, lay=None, flags=0) -> int:
    b = C.c_size_t()
    check(lib().r1s_mat_size(nx, ny, Lv, C.byref(lay) if lay is not None else None, flags,
                             C.byref(b)))
    return b.value


def r1s_mat_init(nx, ny, Lv, lay, flags, values, mem, stream=None):
    h = C.c_void_p()
    lay = lay if lay is not None else layout()
    ins = _inputs(values, nx, ny, Lv, lay)
    check(lib().r1s_mat_init(nx, ny, Lv, C.byref(lay), flags, C.byref(ins), _ptr(mem),
                             mem.numel(), _stream(stream), C.byref(h)))
    return h


def r1s_mat_update(h, values, nx, ny, Lv, lay, stream=None):
    ins = _inputs(values, nx, ny, Lv, lay)
    check(lib().r1s_mat_update(h, C.byref(ins), _stream(stream)))


def _host_i32(a):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(C.c_void_p)


def _graph_shapes(N, n_off, Lv, lay):
    m = Lv + 3
    return {"s_diag": (N, m), "s_sub": (N, Lv - 1), "s_sup": (N, Lv - 1), "s_flow": (N, 6),
            "s_band": (N, 2 * (lay.band - 1), Lv), "s_lev_flow": (N, _slots(lay), Lv),
            "s_flow_lev": (N, _slots(lay), Lv), "s_nbr": (n_off, m), "u_diag": (N, lay.r_diag, m),
            "v_diag": (N, lay.r_diag, m), "u_off": (n_off, lay.r_off, m),
            "v_off": (n_off, lay.r_off, m)}


def _graph_used(lay, L_levels, n_off):
    used = ["s_diag", "s_flow", "u_diag", "v_diag"]
    if L_levels > 1:
        used += ["s_sub", "s_sup"]
    if lay.band > 1:
        used += ["s_band"]
    if lay.arrow:
        used += ["s_lev_flow", "s_flow_lev"]
    if n_off > 0:
        used += ["s_nbr"] + (["u_off", "v_off"] if lay.r_off > 0 else [])
    return used


def _graph_inputs(values, N, n_off, Lv, lay):
    shapes = _graph_shapes(N, n_off, Lv, lay)
    ins = L.GraphInputs()
    for k in _graph_used(lay, Lv, n_off):
        t = values[k]
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
            raise TypeError(f"{k} must be a float64 CUDA tensor")
        if tuple(t.shape) != shapes[k] or not t.is_contiguous():
            raise ValueError(f"{k} must be contiguous with shape {shapes[k]}")
        setattr(ins, k, _ptr(t).value)
    return ins


def r1s_mat_size_graph(n_cells, Lv, lay, indptr, indices, flags=0) -> int:
    b = C.c_size_t()
    ip, pip = _host_i32(indptr)
    ix, pix = _host_i32(indices)
    check(lib().r1s_mat_size_graph(n_cells, Lv, C.byref(lay), pip, pix, flags, C.byref(b)))
    return b.value


def r1s_mat_init_graph(n_cells, Lv, lay, indptr, indices, flags, values, mem, stream=None):
    h = C.c_void_p()
    ip, pip = _host_i32(indptr)
    ix, pix = _host_i32(indices)
    ins = _graph_inputs(values, n_cells, len(ix) - n_cells, Lv, lay)
    check(lib().r1s_mat_init_graph(n_cells, Lv, C.byref(lay), pip, pix, flags, C.byref(ins),
                                   _ptr(mem), mem.numel(), _stream(stream), C.byref(h)))
    return h


def r1s_mat_update_graph(h, values, n_cells, n_off, Lv, lay, stream=None):
    ins = _graph_inputs(values, n_cells, n_off, Lv, lay)
    check(lib().r1s_mat_update_graph(h, C.byref(ins), _stream(stream)))


def r1s_grad_graph(h, nrhs, lam, x, out: Dict[str, torch.Tensor], stream=None):
    g = L.GraphGrads()
    for k in out:
        setattr(g, k, _ptr(out[k]).value)
    check(lib().r1s_grad_graph(h, nrhs, _ptr(lam), _ptr(x), C.byref(g), _stream(stream)))


def _pattern_inputs(values, N, m, nnz, lay, cls=L.PatternInputs):
    P = lay.r_diag + 4 * lay.r_off
    shapes = {"s_cc": (N, nnz), "s_nbr": (N, 4, m), "u": (N, P, m), "v": (N, P, m)}
    ins = cls()
    for k in L.PATTERN_INPUT_FIELDS:
        t = values[k]
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
            raise TypeError(f"{k} must be a float64 CUDA tensor")
        if tuple(t.shape) != shapes[k] or not t.is_contiguous():
            raise ValueError(f"{k} must be contiguous with shape {shapes[k]}")
        setattr(ins, k, _ptr(t).value)
    return ins


def r1s_mat_size_pattern(nx, ny, Lv, lay, indptr, indices, flags=0) -> int:
    b = C.c_size_t()
    ip, pip = _host_i32(indptr)
    ix, pix = _host_i32(indices)
    check(lib().r1s_mat_size_pattern(nx, ny, Lv, C.byref(lay), pip, pix, flags, C.byref(b)))
    return b.value


def r1s_mat_init_pattern(nx, ny, Lv, lay, indptr, indices, flags, values, mem, stream=None):
    h = C.c_void_p()
    ip, pip = _host_i32(indptr)
    ix, pix = _host_i32(indices)
    ins = _pattern_inputs(values, nx * ny, Lv + 3, len(ix), lay)
    check(lib().r1s_mat_init_pattern(nx, ny, Lv, C.byref(lay), pip, pix, flags, C.byref(ins),
                                     _ptr(mem), mem.numel(), _stream(stream), C.byref(h)))
    return h


def r1s_mat_update_pattern(h, values, nx, ny, Lv, nnz, lay, stream=None):
    ins = _pattern_inputs(values, nx * ny, Lv + 3, nnz, lay)
    check(lib().r1s_mat_update_pattern(h, C.byref(ins), _stream(stream)))


def r1s_grad_pattern(h, nrhs, lam, x, out: Dict[str, torch.Tensor], stream=None):
    g = L.PatternGrads()
    for k in out:
        setattr(g, k, _ptr(out[k]).value)
    check(lib().r1s_grad_pattern(h, nrhs, _ptr(lam), _ptr(x), C.byref(g), _stream(stream)))


def r1s_mat_storage(h) -> dict:
    s = L.Storage()
    check(lib().r1s_mat_storage(h, C.byref(s)))
    return {k: getattr(s, k) for k, _ in L.Storage._fields_}


def r1s_matvec(h, precision, trans, nrhs, x, y, stream=None):
    check(lib().r1s_matvec(h, precision, int(trans), nrhs, _ptr(x), _ptr(y), _stream(stream)))


def r1s_residual(h, nrhs, b, x, r, stream=None):
    check(lib().r1s_residual(h, nrhs, _ptr(b), _ptr(x), _ptr(r), _stream(stream)))


def r1s_prec_size(h, flags=0) -> int:
    b = C.c_size_t()
    check(lib().r1s_prec_size(h, flags, C.byref(b)))
    return b.value


def r1s_prec_setup(h, flags, mem, stream=None):
    p = C.c_void_p()
    check(lib().r1s_prec_setup(h, flags, _ptr(mem), mem.numel(), _stream(stream), C.byref(p)))
    return p


def r1s_prec_apply(p, precision, trans, nrhs, r, z, stream=None):
    check(lib().r1s_prec_apply(p, precision, int(trans), nrhs, _ptr(r), _ptr(z), _stream(stream)))


def r1s_matvec_prec(h, p, precision, nrhs, x, y, z, stream=None):
    check(lib().r1s_matvec_prec(h, p, precision, nrhs, _ptr(x), _ptr(y), _ptr(z), _stream(stream)))


def r1s_bsr_size(h) -> int:
    b = C.c_size_t()
    check(lib().r1s_bsr_size(h, C.byref(b)))
    return b.value


def r1s_bsr_init(h, mem, stream=None):
    p = C.c_void_p()
    check(lib().r1s_bsr_init(h, _ptr(mem), mem.numel(), _stream(stream), C.byref(p)))
    return p


def r1s_bsr_matvec(bh, nrhs, x, y, stream=None):
    check(lib().r1s_bsr_matvec(bh, nrhs, _ptr(x), _ptr(y), _stream(stream)))


def r1s_bsr_prec_size(bh) -> int:
    b = C.c_size_t()
    check(lib().r1s_bsr_prec_size(bh, C.byref(b)))
    return b.value


def r1s_bsr_prec_setup(bh, mem, stream=None):
    p = C.c_void_p()
    check(lib().r1s_bsr_prec_setup(bh, _ptr(mem), mem.numel(), _stream(stream), C.byref(p)))
    return p


def r1s_gmres_work_size(h, opts: "L.GmresOpts", nrhs) -> int:
    b = C.c_size_t()
    check(lib().r1s_gmres_work_size(h, C.byref(opts), nrhs, C.byref(b)))
    return b.value


def r1s_gmres(h, bh, p, opts, nrhs, b, x, work, stream=None):
    stats = (L.GmresStats * nrhs)()
    rc = lib().r1s_gmres(h, bh, p, C.byref(opts), nrhs, _ptr(b), _ptr(x), _ptr(work),
                         work.numel(), stats, _stream(stream))
    return rc, [{k: getattr(s, k) for k, _ in L.GmresStats._fields_} for s in stats]


def r1s_gmres_noalloc_size(h, opts: "L.GmresOpts", nrhs) -> int:
    b = C.c_size_t()
    check(lib().r1s_gmres_noalloc_size(h, C.byref(opts), nrhs, C.byref(b)))
    return b.value


def r1s_gmres_noalloc(h, bh, p, opts, nrhs, b, x, stream=None):
    stats = (L.GmresStats * nrhs)()
    rc = lib().r1s_gmres_noalloc(h, bh, p, C.byref(opts), nrhs, _ptr(b), _ptr(x), stats,
                                 _stream(stream))
    return rc, [{k: getattr(s, k) for k, _ in L.GmresStats._fields_} for s in stats]


def r1s_grad(h, nrhs, lam, x, out: Dict[str, torch.Tensor], stream=None):
    g = L.Grads()
    for k in out:
        setattr(g, k, _ptr(out[k]).value)
    check(lib().r1s_grad(h, nrhs, _ptr(lam), _ptr(x), C.byref(g), _stream(stream)))


# -------------------------------------------------------------- classes ---
def _release(obj, destroy):
    """Destroy obj.h through the library handle the object took at creation
    (at interpreter exit the module's own state may already be gone)."""
    h = getattr(obj, "h", None)
    if h is None or not h.value:
        return
    handle = getattr(obj, "_lib", None)
    if handle is None:
        return
    getattr(handle, destroy)(h)
    obj.h = None


class R1Matrix:
    """Structured block r1-sparse Jacobian on one GPU (packed, caller memory).

    ranks = (r_diag, r_off): rank-one pairs of every diagonal / neighbour
    block; u and v have shape [N, r_diag + 4 r_off, m].  band (level-band
    half-width of the diagonal block) and arrow (level/flow coupling) select
    the wide diagonal-block pattern and its arrays s_band, s_lev_flow,
    s_flow_lev."""

    def __init__(self, nx, ny, L_levels, values: Dict[str, torch.Tensor], keep_f32=False,
                 stream=None, ranks=(1, 1), band=1, arrow=False):
        self.nx, self.ny, self.L = nx, ny, L_levels
        self.m = L_levels + 3
        self.N = nx * ny
        self.n = self.N * self.m
        self.r_diag, self.r_off = (int(r) for r in ranks)
        self.n_pairs = self.r_diag + 4 * self.r_off
        self.band, self.arrow = int(band), int(arrow)
        self.layout = layout(self.r_diag, self.r_off, self.band, self.arrow)
        self.flags = L.R1S_KEEP_F32 if keep_f32 else 0
        dev = values["s_diag"].device
        self.device = dev
        self._lib = lib()
        self.mem = _buffer(r1s_mat_size(nx, ny, L_levels, self.layout, self.flags), dev)
        self.h = r1s_mat_init(nx, ny, L_levels, self.layout, self.flags, values, self.mem,
                              stream)

    def __del__(self, _release=_release):  # bound now: module globals are gone at exit
        _release(self, "r1s_mat_destroy")

    def update(self, values, stream=None):
        r1s_mat_update(self.h, values, self.nx, self.ny, self.L, self.layout, stream)

    def storage(self):
        return r1s_mat_storage(self.h)

    def matvec(self, x, trans=False, precision="f64", out=None, stream=None):
        nrhs = _need_vec(x, "x", self.n)
        y = torch.empty_like(x) if out is None else out
        _need_vec(y, "out", self.n)
        prec = L.R1S_F32 if precision == "f32" else L.R1S_F64
        r1s_matvec(self.h, prec, trans, nrhs, x, y, stream)
        return y

    def residual(self, b, x, out=None, stream=None):
        nrhs = _need_vec(b, "b", self.n)
        _need_vec(x, "x", self.n)
        r = torch.empty_like(b) if out is None else out
        r1s_residual(self.h, nrhs, b, x, r, stream)
        return r


class R1GraphMatrix(R1Matrix):
    """The block r1-sparse Jacobian on a general mesh: block structure from
    BR1-BSR style index arrays (block_indptr, block_indices; host arrays),
    values in the general-mesh layout (see gen.make_graph_problem)."""

    def __init__(self, indptr, indices, L_levels, values: Dict[str, torch.Tensor],
                 keep_f32=False, stream=None, ranks=(1, 1), band=1, arrow=False):
        import numpy as np
        self.indptr = np.asarray(indptr, dtype=np.int32)
        self.indices = np.asarray(indices, dtype=np.int32)
        N = len(self.indptr) - 1
        self.nx, self.ny, self.L = N, 1, L_levels
        self.m = L_levels + 3
        self.N = N
        self.n = N * self.m
        self.n_off = len(self.indices) - N
        self.r_diag, self.r_off = (int(r) for r in ranks)
        self.band, self.arrow = int(band), int(arrow)
        self.layout = layout(self.r_diag, self.r_off, self.band, self.arrow)
        self.flags = L.R1S_KEEP_F32 if keep_f32 else 0
        dev = values["s_diag"].device
        self.device = dev
        self._lib = lib()
        self.mem = _buffer(r1s_mat_size_graph(N, L_levels, self.layout, self.indptr, self.indices,
                                              self.flags), dev)
        self.h = r1s_mat_init_graph(N, L_levels, self.layout, self.indptr, self.indices,
                                    self.flags, values, self.mem, stream)

    def update(self, values, stream=None):
        r1s_mat_update_graph(self.h, values, self.N, self.n_off, self.L, self.layout, stream)


class R1PatternMatrix(R1Matrix):
    """The block r1-sparse Jacobian on the structured mesh with a general
    pattern of the diagonal block shared by every cell: pattern = (indptr,
    indices), a CSR pattern over the m = L + 3 unknowns (host arrays);
    values s_cc [N, nnz] in the pattern's entry order, s_nbr, u, v as for
    R1Matrix (see gen.make_pattern_problem)."""

    def __init__(self, nx, ny, L_levels, pattern, values: Dict[str, torch.Tensor], keep_f32=False,
                 stream=None, ranks=(1, 1)):
        import numpy as np
        self.indptr = np.asarray(pattern[0], dtype=np.int32)
        self.indices = np.asarray(pattern[1], dtype=np.int32)
        self.nnz = len(self.indices)
        self.nx, self.ny, self.L = nx, ny, L_levels
        self.m = L_levels + 3
        self.N = nx * ny
        self.n = self.N * self.m
        self.r_diag, self.r_off = (int(r) for r in ranks)
        self.n_pairs = self.r_diag + 4 * self.r_off
        self.band, self.arrow = 1, 0
        self.layout = layout(self.r_diag, self.r_off, 1, 0)
        self.flags = L.R1S_KEEP_F32 if keep_f32 else 0
        dev = values["s_cc"].device
        self.device = dev
        self._lib = lib()
        self.mem = _buffer(r1s_mat_size_pattern(nx, ny, L_levels, self.layout, self.indptr,
                                                self.indices, self.flags), dev)
        self.h = r1s_mat_init_pattern(nx, ny, L_levels, self.layout, self.indptr, self.indices,
                                      self.flags, values, self.mem, stream)

    def update(self, values, stream=None):
        r1s_mat_update_pattern(self.h, values, self.nx, self.ny, self.L, self.nnz, self.layout,
                               stream)


class SMWPreconditioner:
    """Block-Jacobi through the Sherman-Morrison-Woodbury identity."""

    def __init__(self, A: R1Matrix, keep_f32=False, with_trans=False, stream=None):
        self.A = A
        self.flags = (L.R1S_KEEP_F32 if keep_f32 else 0) | (L.R1S_WITH_TRANS if with_trans else 0)
        self._lib = lib()
        self.mem = _buffer(r1s_prec_size(A.h, self.flags), A.device)
        self.h = r1s_prec_setup(A.h, self.flags, self.mem, stream)

    def __del__(self, _release=_release):  # bound now: module globals are gone at exit
        _release(self, "r1s_prec_destroy")

    def apply(self, r, trans=False, precision="f64", out=None, stream=None):
        nrhs = _need_vec(r, "r", self.A.n)
        z = torch.empty_like(r) if out is None else out
        prec = L.R1S_F32 if precision == "f32" else L.R1S_F64
        r1s_prec_apply(self.h, prec, trans, nrhs, r, z, stream)
        return z

    def apply_after_matvec(self, x, precision="f64", out_y=None, out_z=None, stream=None):
        """(y, z) with y = J x and z = M y (the left-preconditioned operator
        M J), computed by one fused kernel where the layout allows."""
        nrhs = _need_vec(x, "x", self.A.n)
        y = torch.empty_like(x) if out_y is None else out_y
        z = torch.empty_like(x) if out_z is None else out_z
        prec = L.R1S_F32 if precision == "f32" else L.R1S_F64
        r1s_matvec_prec(self.A.h, self.h, prec, nrhs, x, y, z, stream)
        return y, z


class BSRMatrix:
    """Dense-block BSR copy of an R1Matrix (the quadratic-in-m baseline)."""

    def __init__(self, A: R1Matrix, stream=None):
        self.A = A
        self._lib = lib()
        self.mem = _buffer(r1s_bsr_size(A.h), A.device)
        self.h = r1s_bsr_init(A.h, self.mem, stream)

    def __del__(self, _release=_release):  # bound now: module globals are gone at exit
        _release(self, "r1s_bsr_destroy")

    def matvec(self, x, out=None, stream=None):
        nrhs = _need_vec(x, "x", self.A.n)
        y = torch.empty_like(x) if out is None else out
        r1s_bsr_matvec(self.h, nrhs, x, y, stream)
        return y


class DenseLUPreconditioner:
    """Classical block-Jacobi: LU with partial pivoting of each dense block."""

    def __init__(self, B: BSRMatrix, stream=None):
        self.B = B
        self.A = B.A
        self._lib = lib()
        self.mem = _buffer(r1s_bsr_prec_size(B.h), B.A.device)
        self.h = r1s_bsr_prec_setup(B.h, self.mem, stream)

    def __del__(self, _release=_release):  # bound now: module globals are gone at exit
        _release(self, "r1s_prec_destroy")

    def apply(self, r, out=None, stream=None):
        nrhs = _need_vec(r, "r", self.A.n)
        z = torch.empty_like(r) if out is None else out
        r1s_prec_apply(self.h, L.R1S_F64, False, nrhs, r, z, stream)
        return z


@dataclass
class GmresResult:
    x: torch.Tensor
    stats: List[dict]
    status: int

    @property
    def converged(self):
        return self.status == L.R1S_OK


def gmres(A: R1Matrix, M, b, x0=None, restart=50, rtol=1e-10, max_cycles=200, trans=False,
          op="structured", B: Optional[BSRMatrix] = None, mode="f64", inner_rtol=1e-5,
          max_outer=10, ortho="delayed", raise_on_noconv=True, work=None,
          noalloc=False, stream=None) -> GmresResult:
    """Restarted right-preconditioned GMRES through r1s_gmres.  ortho: the
    Gram-Schmidt second pass, "delayed" (merged with the next step's first:
    one reduction per step), "selective" or "cgs2" (every step).
    noalloc: solve through r1s_gmres_noalloc (the library's fixed workspace;
    no work buffer is allocated)."""
    orthos = {"selective": L.R1S_ORTHO_SELECTIVE, "cgs2": L.R1S_ORTHO_CGS2,
              "delayed": L.R1S_ORTHO_DELAYED}
    if ortho not in orthos:
        raise ValueError(f"ortho must be one of {sorted(orthos)}")
    nrhs = _need_vec(b, "b", A.n)
    opts = L.GmresOpts(restart=restart, max_cycles=max_cycles, rtol=rtol, trans=int(trans),
                       x0_given=int(x0 is not None),
                       op=L.R1S_OP_BSR if op == "bsr" else L.R1S_OP_STRUCTURED,
                       mode=L.R1S_MODE_MIXED_IR if mode == "mixed" else L.R1S_MODE_F64,
                       inner_rtol=inner_rtol, max_outer=max_outer,
                       ortho=orthos[ortho])
    x = torch.empty_like(b) if x0 is None else x0.clone()
    bh = B.h if B is not None else C.c_void_p(0)
    if noalloc:
        rc, stats = r1s_gmres_noalloc(A.h, bh, M.h, opts, nrhs, b, x, stream)
    else:
        need = r1s_gmres_work_size(A.h, opts, nrhs)
        if work is None or work.numel() < need:
            work = _buffer(need, A.device)
        rc, stats = r1s_gmres(A.h, bh, M.h, opts, nrhs, b, x, work, stream)
    if rc != L.R1S_OK and (raise_on_noconv or rc != L.R1S_ERR_NOCONV):
        raise R1SError(rc, r1s_last_error())
    return GmresResult(x, stats, rc)


def grad(A: R1Matrix, lam, x, stream=None) -> Dict[str, torch.Tensor]:
    """Gradients w.r.t. the structured arrays given lambda = J^{-T} dLoss/dx."""
    nrhs = _need_vec(lam, "lambda", A.n)
    _need_vec(x, "x", A.n)
    if isinstance(A, R1PatternMatrix):
        P = A.r_diag + 4 * A.r_off
        shapes = {"s_cc": (A.N, A.nnz), "s_nbr": (A.N, 4, A.m), "u": (A.N, P, A.m),
                  "v": (A.N, P, A.m)}
        out = {k: torch.empty(shapes[k], dtype=torch.float64, device=A.device)
               for k in L.PATTERN_INPUT_FIELDS}
        r1s_grad_pattern(A.h, nrhs, lam, x, out, stream)
        return out
    if isinstance(A, R1GraphMatrix):
        shapes = _graph_shapes(A.N, A.n_off, A.L, A.layout)
        out = {k: torch.empty(shapes[k], dtype=torch.float64, device=A.device)
               for k in _graph_used(A.layout, A.L, A.n_off)}
        r1s_grad_graph(A.h, nrhs, lam, x, out, stream)
        return out
    shapes = _shapes(A.nx, A.ny, A.L, A.layout)
    out = {k: torch.empty(shapes[k], dtype=torch.float64, device=A.device)
           for k in _used_fields(A.layout)}
    r1s_grad(A.h, nrhs, lam, x, out, stream)
    return out
