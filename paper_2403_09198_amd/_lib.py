"""ctypes declarations of libr1s.so (the C ABI in include/r1s.h).

Loads the in-tree shared library; raises if it has not been built.  There is
no CPU fallback anywhere in the package.
"""
import ctypes as C
import os

# the in-tree build; R1S_LIB may name another build of the same library
LIB_PATH = os.environ.get("R1S_LIB") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libr1s.so")

R1S_OK = 0
R1S_ERR_ARG = -1
R1S_ERR_ALLOC = -2
R1S_ERR_HIP = -3
R1S_ERR_SINGULAR = -4
R1S_ERR_NOCONV = -5
R1S_ERR_NONFINITE = -6
R1S_ERR_UNSUPPORTED = -7
ERROR_NAMES = {
    R1S_ERR_ARG: "R1S_ERR_ARG", R1S_ERR_ALLOC: "R1S_ERR_ALLOC", R1S_ERR_HIP: "R1S_ERR_HIP",
    R1S_ERR_SINGULAR: "R1S_ERR_SINGULAR", R1S_ERR_NOCONV: "R1S_ERR_NOCONV",
    R1S_ERR_NONFINITE: "R1S_ERR_NONFINITE", R1S_ERR_UNSUPPORTED: "R1S_ERR_UNSUPPORTED",
}

R1S_F64, R1S_F32 = 0, 1
R1S_KEEP_F32, R1S_WITH_TRANS = 1, 2
R1S_MAX_M = 256
R1S_MAX_BAND = 8
R1S_MAX_NBR = 8
R1S_OP_STRUCTURED, R1S_OP_BSR = 0, 1
R1S_MODE_F64, R1S_MODE_MIXED_IR = 0, 1
R1S_ORTHO_DELAYED, R1S_ORTHO_SELECTIVE, R1S_ORTHO_CGS2 = 0, 1, 2
R1S_NOALLOC_MAX_BYTES = 64 << 20


INPUT_FIELDS = ("s_diag", "s_sub", "s_sup", "s_flow", "s_nbr", "u", "v", "s_band", "s_lev_flow",
                "s_flow_lev")


class Layout(C.Structure):
    _fields_ = [("r_diag", C.c_int), ("r_off", C.c_int), ("band", C.c_int), ("arrow", C.c_int)]


class Inputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in INPUT_FIELDS]


class Grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in INPUT_FIELDS]


GRAPH_INPUT_FIELDS = ("s_diag", "s_sub", "s_sup", "s_flow", "s_band", "s_lev_flow", "s_flow_lev",
                      "s_nbr", "u_diag", "v_diag", "u_off", "v_off")


class GraphInputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in GRAPH_INPUT_FIELDS]


class GraphGrads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in GRAPH_INPUT_FIELDS]


PATTERN_INPUT_FIELDS = ("s_cc", "s_nbr", "u", "v")


class PatternInputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in PATTERN_INPUT_FIELDS]


class PatternGrads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in PATTERN_INPUT_FIELDS]


class Storage(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_cells", "n_blocks", "m", "structured_values", "structured_padded", "bsr_values",
        "index_bytes", "matvec_bytes", "smw_apply_bytes")]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_cycles", C.c_int), ("rtol", C.c_double),
                ("trans", C.c_int), ("x0_given", C.c_int), ("op", C.c_int), ("mode", C.c_int),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int), ("ortho", C.c_int)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("outer", C.c_int),
                ("converged", C.c_int), ("rel_residual", C.c_double)]


_VP = C.c_void_p
_I = C.c_int
_SZ = C.c_size_t
_PSZ = C.POINTER(C.c_size_t)

# name -> (restype, argtypes); every function declared in include/r1s.h
SIGNATURES = {
    "r1s_last_error": (C.c_char_p, []),
    "r1s_mat_size": (_I, [_I, _I, _I, C.POINTER(Layout), _I, _PSZ]),
    "r1s_mat_init": (_I, [_I, _I, _I, C.POINTER(Layout), _I, C.POINTER(Inputs), _VP, _SZ, _VP,
                          C.POINTER(_VP)]),
    "r1s_mat_update": (_I, [_VP, C.POINTER(Inputs), _VP]),
    "r1s_mat_destroy": (_I, [_VP]),
    "r1s_mat_size_graph": (_I, [_I, _I, C.POINTER(Layout), _VP, _VP, _I, _PSZ]),
    "r1s_mat_init_graph": (_I, [_I, _I, C.POINTER(Layout), _VP, _VP, _I, C.POINTER(GraphInputs),
                                _VP, _SZ, _VP, C.POINTER(_VP)]),
    "r1s_mat_update_graph": (_I, [_VP, C.POINTER(GraphInputs), _VP]),
    "r1s_mat_size_pattern": (_I, [_I, _I, _I, C.POINTER(Layout), _VP, _VP, _I, _PSZ]),
    "r1s_mat_init_pattern": (_I, [_I, _I, _I, C.POINTER(Layout), _VP, _VP, _I,
                                  C.POINTER(PatternInputs), _VP, _SZ, _VP, C.POINTER(_VP)]),
    "r1s_mat_update_pattern": (_I, [_VP, C.POINTER(PatternInputs), _VP]),
    "r1s_mat_storage": (_I, [_VP, C.POINTER(Storage)]),
    "r1s_matvec": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "r1s_residual": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "r1s_prec_size": (_I, [_VP, _I, _PSZ]),
    "r1s_prec_setup": (_I, [_VP, _I, _VP, _SZ, _VP, C.POINTER(_VP)]),
    "r1s_prec_apply": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "r1s_matvec_prec": (_I, [_VP, _VP, _I, _I, _VP, _VP, _VP, _VP]),
    "r1s_prec_destroy": (_I, [_VP]),
    "r1s_bsr_size": (_I, [_VP, _PSZ]),
    "r1s_bsr_init": (_I, [_VP, _VP, _SZ, _VP, C.POINTER(_VP)]),
    "r1s_bsr_matvec": (_I, [_VP, _I, _VP, _VP, _VP]),
    "r1s_bsr_prec_size": (_I, [_VP, _PSZ]),
    "r1s_bsr_prec_setup": (_I, [_VP, _VP, _SZ, _VP, C.POINTER(_VP)]),
    "r1s_bsr_destroy": (_I, [_VP]),
    "r1s_gmres_work_size": (_I, [_VP, C.POINTER(GmresOpts), _I, _PSZ]),
    "r1s_gmres": (_I, [_VP, _VP, _VP, C.POINTER(GmresOpts), _I, _VP, _VP, _VP, _SZ,
                       C.POINTER(GmresStats), _VP]),
    "r1s_gmres_noalloc_size": (_I, [_VP, C.POINTER(GmresOpts), _I, _PSZ]),
    "r1s_gmres_noalloc": (_I, [_VP, _VP, _VP, C.POINTER(GmresOpts), _I, _VP, _VP,
                               C.POINTER(GmresStats), _VP]),
    "r1s_grad": (_I, [_VP, _I, _VP, _VP, C.POINTER(Grads), _VP]),
    "r1s_grad_graph": (_I, [_VP, _I, _VP, _VP, C.POINTER(GraphGrads), _VP]),
    "r1s_grad_pattern": (_I, [_VP, _I, _VP, _VP, C.POINTER(PatternGrads), _VP]),
}

_lib = None


class R1SError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded libr1s.so with argtypes set (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2403_09198_amd.csrc.build` (no CPU fallback exists)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(rc):
    if rc != R1S_OK:
        raise R1SError(rc, lib().r1s_last_error().decode())
    return rc
