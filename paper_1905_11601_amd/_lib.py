"""ctypes loader for the in-tree HIP library libfvk.so (built by build.py).

Argument marshalling only: every operation runs in the library's HIP kernels.
There is no fallback: if the library is missing or fails to load, importing
the binding raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvk.so")

c_int, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
c_char_p = ctypes.c_char_p
P = ctypes.POINTER

STATUS = {0: "FVK_OK", 1: "FVK_EINVAL", 2: "FVK_ENOMEM", 3: "FVK_EHIP", 4: "FVK_ENOCONV",
          5: "FVK_EBREAKDOWN"}


class NewtonOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("gmres_m", c_int), ("gmres_max_restarts", c_int),
                ("sat_ratio", c_double), ("bicgstab_max_it", c_int), ("lin_tol", c_double),
                ("max_newton", c_int)]


class NewtonReport(ctypes.Structure):
    _fields_ = [("res_before", c_double), ("res_after", c_double), ("newton_its", c_int),
                ("gmres_cycles", c_int), ("bicgstab_its", c_int), ("krylov_vecs", c_int),
                ("lin_rel_res", c_double), ("lin_status", c_int)]


# name -> (restype, argtypes); every function declared in include/fvk.h
SIGNATURES = {
    "fvk_create": (c_int, [P(c_void_p), c_int, c_int, c_int, c_int, c_double, c_int, c_double,
                           c_double, c_int, c_void_p]),
    "fvk_destroy": (c_int, [c_void_p]),
    "fvk_set_stream": (c_int, [c_void_p, c_void_p]),
    "fvk_set_params": (c_int, [c_void_p, c_double, c_double]),
    "fvk_set_coeffs": (c_int, [c_void_p, c_double, c_double, c_double]),
    "fvk_set_terms": (c_int, [c_void_p, c_int]),
    "fvk_set_shift": (c_int, [c_void_p, c_double]),
    "fvk_get_shift": (c_int, [c_void_p, P(c_double)]),
    "fvk_set_precision": (c_int, [c_void_p, c_int]),
    "fvk_set_tpf_path": (c_int, [c_void_p, c_int]),
    "fvk_get_tpf_path": (c_int, [c_void_p, P(c_int)]),
    "fvk_set_simple": (c_int, [c_void_p, c_double, c_int]),
    "fvk_layout": (c_int, [c_void_p, P(c_size_t), P(c_size_t), P(c_size_t)]),
    "fvk_grid_axis": (c_int, [c_void_p, c_int, P(c_double), P(c_double), P(c_double)]),
    "fvk_last_error": (c_char_p, [c_void_p]),
    "fvk_tridiag_eig": (c_int, [c_int, P(c_double), P(c_double), P(c_double), P(c_double)]),
    "fv_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "fv_jacvec": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "fvk_project": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "simple_krylov_vec": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                  P(c_int), P(c_double)]),
    "fvk_mixed_passes": (c_int, [c_void_p, P(c_int), P(c_int)]),
    "fvk_psi_projection": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "fvk_simple_stats": (c_int, [c_void_p, P(c_double), P(c_int)]),
    "arnoldi_step": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int, P(c_double), c_int]),
    "arnoldi_step_lagged": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int, P(c_double),
                                    c_int, c_int]),
    "arnoldi_step_lagged_applied": (c_int, [c_void_p, c_void_p, c_size_t, c_int, P(c_double),
                                            c_int]),
    "fvk_lincomb3": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_double, c_void_p,
                             c_double, c_size_t]),
    "arnoldi_finish": (c_int, [c_void_p, c_void_p, c_size_t, c_int, P(c_double), c_int]),
    "fvk_set_timing": (c_int, [c_void_p, c_int]),
    "fvk_timing_read": (c_int, [c_void_p, P(c_double), P(c_int)]),
    "fvk_multidot": (c_int, [c_void_p, c_void_p, c_size_t, c_int, c_void_p, c_size_t,
                             P(c_double)]),
    "fvk_multidot_noalloc": (c_int, [c_void_p, c_void_p, c_size_t, c_int, c_void_p, c_size_t,
                                     c_void_p]),
    "fvk_multiaxpy": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_size_t, c_int,
                              P(c_double), c_size_t]),
    "fvk_axpby": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_double, c_size_t]),
    "fvk_basis_rotate": (c_int, [c_void_p, c_void_p, c_size_t, c_int, P(c_double), c_int,
                                 c_size_t]),
    "fvk_newton_defaults": (None, [P(NewtonOpts)]),
    "newton_step": (c_int, [c_void_p, c_void_p, P(NewtonOpts), P(NewtonReport)]),
    "fvk_linear_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, P(NewtonOpts),
                                 P(NewtonReport)]),
}

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_1905_11601_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
