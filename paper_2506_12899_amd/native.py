"""ctypes binding of libsbm.so (the C ABI in include/sbm.h).

Argument marshalling only: every step of the method runs inside the library.
Torch is used for device memory (tensors are passed by data_ptr()) and for
the stream.  Importing this module does not load the library; `lib()` does,
and raises if it has not been built -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsbm.so")

SBM_OK, SBM_NOT_CONVERGED = 0, 1
SBM_EINVAL = -1
NOALLOC_SCRATCH_BYTES = 128 << 20     # SBM_NOALLOC_SCRATCH_BYTES in include/sbm.h
GEOM_BALLS, GEOM_STAR2D, GEOM_CALLBACK, GEOM_ELLIPSOID = 0, 1, 2, 3

PHI_FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)
VEC_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)
FIELD_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_longlong, C.POINTER(C.c_double), C.c_void_p)


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("kind", C.c_int), ("n_balls", C.c_int),
                ("centers", C.POINTER(C.c_double)), ("radii", C.POINTER(C.c_double)),
                ("rotation", C.POINTER(C.c_double)),
                ("star_r0", C.c_double), ("star_a", C.c_double), ("star_k", C.c_int),
                ("phi", PHI_FN), ("grad", VEC_FN), ("hess", VEC_FN), ("user", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("c_F", C.c_double), ("c_G", C.c_double),
                ("alpha", C.c_double), ("ext", C.c_int), ("omega", C.c_double),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("coarse_min", C.c_int), ("coarse_dofs", C.c_int),
                ("vcycle_fp32", C.c_int), ("allow_singular", C.c_int), ("fuse_transfers", C.c_int),
                ("penalty_p", C.c_int), ("lambda_frac", C.c_double), ("frac_m", C.c_int), ("min_neighbours", C.c_int), ("stab", C.c_double),
                ("smoother", C.c_int), ("cheb_degree", C.c_int), ("cheb_range", C.c_double),
                ("pencil", C.c_int),
                ("device", C.c_int),
                ("stream", C.c_void_p)]


class Layout(C.Structure):
    _fields_ = [("n_dofs", C.c_longlong), ("n_active", C.c_int), ("n_colour0", C.c_int),
                ("dofs_per_cell", C.c_int), ("n_levels", C.c_int), ("n_boundary_cells", C.c_int),
                ("n_surrogate_faces", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("rel_residual_true", C.c_double),
                ("seconds", C.c_double)]


_LIB = None

# (name, restype, argtypes) of every entry point declared in include/sbm.h
_VP = C.c_void_p
SIGNATURES = [
    ("sbm_default_options", C.c_int, [C.c_int, C.c_int, C.POINTER(Options)]),
    ("sbm_setup", C.c_int, [C.POINTER(Geometry), C.c_int, C.c_int, C.POINTER(Options), C.POINTER(_VP)]),
    ("sbm_layout_info", C.c_int, [_VP, C.POINTER(Layout)]),
    ("sbm_active_cells", C.c_int, [_VP, C.c_int, C.POINTER(C.c_int), C.c_longlong]),
    ("sbm_level_info", C.c_int, [_VP, C.c_int] + [C.POINTER(C.c_int)] * 5),
    ("sbm_level_blocks", C.c_int, [_VP, C.c_int] + [C.POINTER(C.c_int)] * 3),
    ("sbm_shifts", C.c_int, [_VP, C.c_int, C.POINTER(C.c_double), C.c_longlong]),
    ("sbm_set_shifts", C.c_int, [_VP, C.c_int, C.POINTER(C.c_double), C.c_longlong]),
    ("sbm_rhs", C.c_int, [_VP, FIELD_FN, FIELD_FN, _VP, _VP]),
    ("sbm_apply", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("sbm_vcycle", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("sbm_solve", C.c_int, [_VP, _VP, _VP, C.c_double, C.c_int, C.c_int, C.POINTER(Stats)]),
    ("sbm_solve_noalloc", C.c_int, [_VP, _VP, _VP, C.c_double, C.c_int, C.c_int, C.POINTER(Stats)]),
    ("sbm_solve_noalloc_doubles", C.c_longlong, [_VP, C.c_int]),
    ("sbm_level_apply", C.c_int, [_VP, C.c_int, _VP, _VP, C.c_int]),
    ("sbm_colour_update", C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP, C.c_int]),
    ("sbm_restrict", C.c_int, [_VP, C.c_int, _VP, _VP, C.c_int]),
    ("sbm_prolong_add", C.c_int, [_VP, C.c_int, _VP, _VP, C.c_int]),
    ("sbm_cell_block", C.c_int, [_VP, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("sbm_coarse_matrix", C.c_int, [_VP, C.POINTER(C.c_double), C.c_longlong]),
    ("sbm_set_vcycle_fp32", C.c_int, [_VP, C.c_int]),
    ("sbm_feature_dim", C.c_int, [C.c_int]),
    ("sbm_boundary_cells", C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_longlong]),
    ("sbm_boundary_features", C.c_int, [_VP, C.POINTER(C.c_double), C.c_longlong]),
    ("sbm_boundary_samples", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("sbm_collect_pairs", C.c_int, [_VP] * 8),
    ("sbm_richardson", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("sbm_set_learned", C.c_int, [_VP, _VP, C.c_int]),
    ("sbm_set_learned_arrays", C.c_int, [_VP] + [C.POINTER(C.c_double)] * 3),
    ("sbm_use_learned", C.c_int, [_VP, C.c_int]),
    ("sbm_mlp_forward", C.c_int, [C.c_int] * 5 + [_VP] * 6),
    ("sbm_mlp_loss_grad", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double] + [_VP] * 8),
    ("sbm_mlp_work_elems", C.c_longlong, [C.c_int] * 4),
    ("sbm_mlp_backward", C.c_int, [C.c_int] * 5 + [_VP] * 9),
    ("sbm_adam", C.c_int, [C.c_int, _VP, _VP, _VP, _VP, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, _VP]),
    ("sbm_mlp_infer_wbuf_elems", C.c_longlong, [C.c_int]),
    ("sbm_mlp_infer_bf16", C.c_int, [C.c_int] * 4 + [_VP] * 5),
    ("sbm_sync", C.c_int, [_VP]),
    ("sbm_destroy", C.c_int, [_VP]),
    ("sbm_strerror", C.c_char_p, [C.c_int]),
    ("sbm_last_error", C.c_char_p, [_VP]),
]


def lib():
    """Load libsbm.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} not built: run `python -m paper_2506_12899_amd.build`")
        L = C.CDLL(LIBPATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


class SbmError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        text = lib().sbm_strerror(status).decode()
        super().__init__(f"sbm status {status} ({text}){': ' + msg if msg else ''}")


def check(status, handle=None):
    if status < 0:
        msg = lib().sbm_last_error(handle).decode() if handle else ""
        raise SbmError(status, msg)
    return status


def default_options(dim, p):
    o = Options()
    check(lib().sbm_default_options(dim, p, C.byref(o)))
    return o
