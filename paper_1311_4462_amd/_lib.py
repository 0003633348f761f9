"""ctypes declarations of the C ABI in include/tm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

c_int, c_double, c_void_p, c_size_t, c_uint = (ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                                ctypes.c_size_t, ctypes.c_uint)


class TMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tm error {code}: {msg}")
        self.code = code


class tm_params(ctypes.Structure):
    _fields_ = [("dims", c_int * 4), ("kappa", c_double), ("mu", c_double),
                ("epsilon", c_double), ("flavor", c_int), ("t_antiperiodic", c_int),
                ("csw", c_double)]


class tm_cg_params(ctypes.Structure):
    _fields_ = [("pc", c_int), ("tol", c_double), ("maxiter", c_int), ("outer", c_int),
                ("inner", c_int), ("delta", c_double), ("use_x0", c_int), ("nrhs", c_int),
                ("graph_iters", c_int), ("check_every", c_int), ("solution", c_int),
                ("stall_factor", c_double), ("max_stalls", c_int)]


class tm_cg_result(ctypes.Structure):
    _fields_ = [("iters", c_int), ("reliable_updates", c_int),
                ("true_rel_res_normal", c_double), ("true_rel_res_pc", c_double),
                ("seconds", c_double), ("true_rel_res_full", c_double),
                ("precision_fallbacks", c_int), ("history_len", c_int),
                ("res_history", c_double * 16)]


class tm_solve_params(ctypes.Structure):
    _fields_ = [("cg", tm_cg_params), ("solve_type", c_int), ("solution", c_int)]


P = ctypes.POINTER
_SIGS = {
    "tm_error_string": (ctypes.c_char_p, [c_int]),
    "tm_last_error": (ctypes.c_char_p, [c_void_p]),
    "tm_ctx_create": (c_int, [P(c_void_p), c_void_p]),
    "tm_ctx_destroy": (c_int, [c_void_p]),
    "tm_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "tm_set_tuning": (c_int, [c_void_p, c_int]),
    "tm_gauge_create": (c_int, [c_void_p, P(c_void_p), c_void_p, P(tm_params), c_int, c_uint]),
    "tm_gauge_destroy": (c_int, [c_void_p]),
    "tm_gauge_bytes": (c_size_t, [c_void_p, c_int]),
    "tm_spinor_bytes": (c_size_t, [P(tm_params), c_int, c_int]),
    "tm_spinor_pack": (c_int, [c_void_p, c_void_p, c_void_p, P(tm_params), c_int, c_int, c_int,
                               c_int]),
    "tm_spinor_unpack": (c_int, [c_void_p, c_void_p, c_void_p, P(tm_params), c_int, c_int, c_int,
                                 c_int]),
    "tm_dslash": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                          c_int, c_void_p, c_double, c_int]),
    "tm_mat_pc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    "tm_mat_pc_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    "tm_scale": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_double, P(tm_params), c_int]),
    "tm_twist": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "tm_twist_inv": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    "tm_prepare": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int]),
    "tm_reconstruct_odd": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int]),
    "tm_cg": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, P(tm_cg_params), P(tm_cg_result)]),
    "tm_cg_batched": (c_int, [c_void_p, c_int, P(c_void_p), P(c_void_p), P(c_void_p), P(c_int),
                              P(tm_cg_params), P(tm_cg_result)]),
    "tm_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                         P(tm_solve_params), P(tm_cg_result)]),
    "tm_norm2": (c_int, [c_void_p, P(c_double), c_void_p, P(tm_params), c_int, c_int]),
    "tm_dot": (c_int, [c_void_p, P(c_double), c_void_p, c_void_p, P(tm_params), c_int, c_int]),
    "tm_convert": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, P(tm_params), c_int]),
    "tm_force": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int, c_int, c_double,
                         c_int, c_void_p]),
    "tm_plan_hop_lds": (c_int, [c_int, c_int, ctypes.c_uint, ctypes.c_uint, ctypes.c_uint,
                                ctypes.c_uint, P(ctypes.c_uint)]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """The loaded libtm.so.  Raises if the HIP library has not been built:
    there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1311_4462_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
