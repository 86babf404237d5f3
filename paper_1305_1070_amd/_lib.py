"""ctypes binding of libndnegf.so: the C entry points of include/ndnegf.h
under the same names, with argument marshalling only.

The shared library is built in place by paper_1305_1070_amd.build (or
__graft_entry__.build()); importing this module never builds it.  If it is
missing, load() raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libndnegf.so")

NDG_OK = 0
STATUS = {0: "NDG_OK", -1: "NDG_EINVAL", -2: "NDG_ENOTSYM", -3: "NDG_ECONTACT",
          -4: "NDG_ESINGULAR", -5: "NDG_ENOMEM", -6: "NDG_EHIP", -7: "NDG_ENONFINITE",
          -8: "NDG_ENOTSPD"}
NDG_FP64, NDG_MIXED = 0, 1


class NdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class TreeOpts(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("max_cluster", C.c_int32), ("tree_kind", C.c_int32),
                ("slab", C.c_int32), ("layer_max", C.c_int32), ("reserved", C.c_int32),
                ("layer_of", C.POINTER(C.c_int32))]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nclusters", C.c_int32), ("max_height", C.c_int32),
                ("max_cluster", C.c_int32), ("max_boundary", C.c_int32), ("ncontacts", C.c_int32),
                ("reserved", C.c_int32), ("nnz_boundary", C.c_int64),
                ("ops_fold_inv", C.c_double), ("ops_fold_psi", C.c_double),
                ("ops_fold_update", C.c_double), ("ops_gr_off", C.c_double),
                ("ops_gr_diag", C.c_double), ("ops_gl_chain", C.c_double),
                ("ops_gl_off", C.c_double), ("ops_gl_diag", C.c_double),
                ("ops_total", C.c_double), ("ops_rgf_equiv", C.c_double),
                ("workspace_bytes_per_energy", C.c_int64),
                ("scatter_bytes_per_energy", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("height", C.c_int32), ("size_class", C.c_int32),
                ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


P = C.c_void_p


class SolveArgs(C.Structure):
    _fields_ = [("nE", C.c_int32), ("E", C.c_void_p), ("eta", C.c_double), ("V", C.c_void_p),
                ("sig_r", C.POINTER(C.c_void_p)), ("sig_less", C.POINTER(C.c_void_p)),
                ("diag_gr", C.c_void_p), ("diag_gless", C.c_void_p),
                ("diag_ggreater", C.c_void_p), ("growth", C.c_void_p)]


I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
F64P = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "ndg_analyze": (C.c_int, [C.c_int64, I64P, I32P, F64P, C.c_int32, C.POINTER(I32P), I32P, F64P,
                              C.POINTER(TreeOpts), C.POINTER(P)]),
    "ndg_symbolic_destroy": (None, [P]),
    "ndg_symbolic_info": (C.c_int, [P, C.POINTER(Info)]),
    "ndg_symbolic_arrays": (C.c_int, [P, I32P, I32P, I32P, I32P, I64P, I32P]),
    "ndg_plan_create": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(P)]),
    "ndg_plan_destroy": (C.c_int, [P]),
    "ndg_plan_info": (C.c_int, [P, C.POINTER(Info)]),
    "ndg_solve": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), P, P, P,
                            P, C.c_int, P]),
    "ndg_solve_transport": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), P,
                                      P, P, P, P, P]),
    "ndg_plan_status": (C.c_int, [P, I32P, I32P, I32P]),
    "ndg_plan_export_block": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, P]),
    "ndg_density": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), P, P,
                              C.c_int, P]),
    "ndg_plan_enable_adjoint": (C.c_int, [P]),
    "ndg_density_vjp": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), P,
                                  P, P, C.c_int, P]),
    "ndg_density_vjp_noalloc": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P),
                                          P, P, P, C.c_int, P]),
    "ndg_plan_enable_scattering": (C.c_int, [P]),
    "ndg_solve_scattering": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P),
                                       P, P, P, P, P, P, P, P]),
    "ndg_scba": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), C.c_double,
                           C.c_double, C.c_double, C.c_int32, P, P, P, P, P, P, I32P, F64P, P]),
    "ndg_poisson_newton_step": (C.c_int, [P, C.c_int32, P, C.c_double, P, C.POINTER(P), C.POINTER(P), P,
                                          P, P, P, C.c_int64, C.c_double, P, C.c_double, C.c_int32, P,
                                          F64P, I32P, F64P, P]),
    "ndg_plan_set_profiling": (C.c_int, [P, C.c_int32]),
    "ndg_plan_profile": (C.c_int, [P, C.c_int32, C.POINTER(KernelStat), C.POINTER(C.c_int32)]),
    "ndg_symbolic_costs": (C.c_int, [P, C.c_int32, C.POINTER(KernelStat), C.POINTER(C.c_int32)]),
    "ndg_batch_create": (C.c_int, [C.c_int32, C.POINTER(P), C.POINTER(P)]),
    "ndg_batch_destroy": (C.c_int, [P]),
    "ndg_batch_solve": (C.c_int, [P, C.POINTER(SolveArgs), C.c_int, P]),
    "ndg_batch_launches": (C.c_int32, [P]),
    "ndg_status_string": (C.c_char_p, [C.c_int32]),
    "ndg_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str | None = None):
    """Loads the shared library (once) and declares every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    # The library and PyTorch must share one HIP runtime: torch ships its own
    # libamdhip64.so.7, so it is loaded first and the library's dependency on
    # that soname then resolves to the same copy.
    import torch  # noqa: F401
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libndnegf.so not built (%s); run python -m paper_1305_1070_amd.build"
                           % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != NDG_OK:
        msg = load().ndg_last_error()
        raise NdgError(code, msg.decode() if msg else "")
