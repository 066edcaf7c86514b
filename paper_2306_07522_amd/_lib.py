"""ctypes declarations of the C ABI in include/heom.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheom.so")

heom_status = C.c_int32
heom_drive_fn = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.c_void_p)
vp = C.c_void_p
dp = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)
u64p = C.POINTER(C.c_uint64)

HEOM_FP64, HEOM_FP32 = 0, 1
HEOM_BOSON, HEOM_FERMION = 0, 1
HEOM_U_R, HEOM_U_I, HEOM_U_RI = 0, 1, 2
HEOM_PADE, HEOM_MATSUBARA = 0, 1
HEOM_OP_PROPAGATE, HEOM_OP_STEADY, HEOM_OP_SPECTRUM = 0, 1, 2
HEOM_PREC_NONE, HEOM_PREC_JACOBI, HEOM_PREC_NN, HEOM_PREC_SCALED, HEOM_PREC_BLOCK = 0, 1, 2, 3, 4
HEOM_SOLVE_FP64, HEOM_SOLVE_FP32_IR, HEOM_SOLVE_SHIFTED = 0, 1, 2


class heom_bath(C.Structure):
    _fields_ = [("kind", C.c_int32), ("op", dp), ("n_exp", C.c_int32), ("u_type", i32p), ("xi", dp), ("chi", dp),
                ("eta_p", dp), ("gam_p", dp), ("eta_m", dp), ("gam_m", dp)]


class heom_info(C.Structure):
    _fields_ = [("n_ado", C.c_int64), ("d", C.c_int32), ("n_bos_exp", C.c_int32), ("n_ferm_exp", C.c_int32),
                ("m_max", C.c_int32), ("n_max", C.c_int32), ("parity", C.c_int32), ("n_ops", C.c_int32),
                ("n_edges", C.c_int64), ("n_leaf", C.c_int64), ("n_tiers", C.c_int32),
                ("tier_offset", C.c_int64 * 34), ("table_bytes", C.c_int64), ("vector_bytes_fp64", C.c_int64)]


class heom_slab_stats(C.Structure):
    _fields_ = [("built", C.c_int32), ("max_vertices", C.c_int32 * 2), ("children", C.c_int64),
                ("parents", C.c_int64), ("jobs", C.c_int64 * 2), ("entries", C.c_int64 * 2),
                ("cost", C.c_int64 * 2), ("xcd_cost", (C.c_int64 * 8) * 2)]


class heom_solver_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double), ("precond", C.c_int32),
                ("mode", C.c_int32), ("inner_tol", C.c_double), ("max_refine", C.c_int32),
                ("rhs_chunk", C.c_int32), ("nn", vp), ("fallback", C.c_int32), ("use_x0", C.c_int32),
                ("deflate", C.c_int32)]


class heom_solver_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
                ("refinements", C.c_int32), ("fell_back", C.c_int32), ("true_residual", C.c_double),
                ("seconds", C.c_double), ("applies", C.c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "heom_version": (C.c_char_p, []),
    "heom_last_error": (C.c_char_p, []),
    "heom_status_string": (C.c_char_p, [heom_status]),
    "heom_pade_params": (heom_status, [C.c_int32, C.c_int32, C.c_int32, dp, dp]),
    "heom_exponents_lorentz": (heom_status, [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                             dp, dp, dp, dp]),
    "heom_exponents_drude_lorentz": (heom_status, [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, dp, dp]),
    "heom_build_hierarchy": (heom_status, [C.c_int32, dp, C.c_int32, C.POINTER(heom_bath), C.c_int32, C.c_int32,
                                           C.c_int32, dp, C.POINTER(vp)]),
    "heom_build_hierarchy_pruned": (heom_status, [C.c_int32, dp, C.c_int32, C.POINTER(heom_bath), C.c_int32,
                                                  C.c_int32, C.c_int32, dp, C.c_double, C.POINTER(vp)]),
    "heom_free": (None, [vp]),
    "heom_hierarchy_info": (heom_status, [vp, C.POINTER(heom_info)]),
    "heom_hierarchy_ados": (heom_status, [vp, i32p, u64p, i32p]),
    "heom_ado_index": (heom_status, [vp, i32p, i32p, C.c_int32, i64p, i32p]),
    "heom_hierarchy_tables": (heom_status, [vp, dp, i64p, i32p, i32p, i32p, i32p]),
    "heom_apply": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, dp, vp]),
    "heom_apply_shifted": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, vp, vp]),
    "heom_apply_steady_operator": (heom_status, [vp, C.c_int32, vp, vp, vp]),
    "heom_apply_tiled": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, dp, C.c_int32, vp]),
    "heom_apply_plan": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, dp, C.c_int32, vp]),
    "heom_slab_plan_stats": (heom_status, [vp, C.POINTER(heom_slab_stats)]),
    "heom_default_opts": (None, [C.POINTER(heom_solver_opts)]),
    "heom_spectrum_chunk": (C.c_int32, [vp, C.POINTER(heom_solver_opts)]),
    "heom_workspace_size": (heom_status, [vp, C.c_int32, C.POINTER(heom_solver_opts), C.c_int64,
                                          C.POINTER(C.c_size_t)]),
    "heom_propagate": (heom_status, [vp, C.c_int32, vp, C.c_double, C.c_int64, C.c_int64, vp, C.c_int32, vp,
                                     C.c_size_t, vp]),
    "heom_steady": (heom_status, [vp, vp, C.POINTER(heom_solver_opts), C.POINTER(heom_solver_report), vp,
                                  C.c_size_t, vp]),
    "heom_spectrum": (heom_status, [vp, vp, vp, C.c_int32, dp, dp, C.c_int64, dp, C.POINTER(heom_solver_opts),
                                    C.POINTER(heom_solver_report), vp, C.c_size_t, vp]),
    "heom_nn_create": (heom_status, [C.c_int32, C.c_int32, C.c_uint64, C.POINTER(vp)]),
    "heom_nn_free": (None, [vp]),
    "heom_nn_info": (heom_status, [vp, i32p, i32p, i32p]),
    "heom_nn_get_params": (heom_status, [vp, C.POINTER(C.c_float)]),
    "heom_nn_set_params": (heom_status, [vp, C.POINTER(C.c_float)]),
    "heom_nn_save": (heom_status, [vp, C.c_char_p]),
    "heom_nn_load": (heom_status, [C.c_char_p, C.POINTER(vp)]),
    "heom_nn_pairs": (heom_status, [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp]),
    "heom_nn_forward": (heom_status, [vp, vp, C.c_int64, vp, vp]),
    "heom_nn_gradients": (heom_status, [vp, vp, vp, vp, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float), vp]),
    "heom_nn_train": (heom_status, [vp, vp, vp, vp, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                    C.c_uint64, C.POINTER(C.c_float), vp]),
    "heom_steady_residual": (heom_status, [vp, vp, vp, vp]),
    "heom_vector_axpby": (heom_status, [C.c_int32, vp, C.c_double, vp, C.c_double, C.c_int64, vp]),
    "heom_batch_create": (heom_status, [C.c_int32, C.POINTER(vp), C.POINTER(vp)]),
    "heom_batch_free": (None, [vp]),
    "heom_batch_info": (heom_status, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), i32p, i32p]),
    "heom_batch_apply": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, vp]),
    "heom_batch_tune": (heom_status, [vp, C.c_int32, vp, vp, C.c_int32, dp, dp, vp]),
    "heom_batch_shape": (heom_status, [vp, i32p]),
    "heom_prepare": (heom_status, [vp]),
    "heom_batch_set_shape": (heom_status, [vp, i32p]),
    "heom_propagate_driven": (heom_status, [vp, C.c_int32, vp, C.c_double, C.c_double, C.c_int64, C.c_int64, vp,
                                            C.c_int32, dp, heom_drive_fn, vp, vp, C.c_size_t, vp]),
    "heom_hierarchy_set_lindblad": (heom_status, [vp, C.c_int32, dp]),
    "heom_current": (heom_status, [vp, vp, C.c_int32, i32p, dp, vp]),
    "heom_current_noalloc": (heom_status, [vp, vp, C.c_int32, i32p, dp, vp]),
    "heom_precondition": (heom_status, [vp, C.c_int32, C.c_int32, vp, vp, C.c_int32, vp, C.c_int32, vp]),
    "heom_batch_workspace_size": (heom_status, [vp, C.POINTER(heom_solver_opts), C.POINTER(C.c_size_t)]),
    "heom_batch_steady": (heom_status, [vp, vp, C.POINTER(heom_solver_opts), C.POINTER(heom_solver_report),
                                        C.c_int32, vp, C.c_size_t, vp]),
}

_lib = None


class HeomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"heom status {status}: {msg}")
        self.status = status


def _hip_runtimes():
    """Paths of the libamdhip64 copies mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def load():
    """Load libheom.so (built in-tree by build_lib.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2306_07522_amd/build_lib.py")
    # The binding hands the library torch's device pointers and streams, which
    # are only valid inside the HIP runtime that torch loaded.  Importing torch
    # first makes the dynamic linker resolve libheom's libamdhip64.so.7 to that
    # same copy; loading libheom first would map a second runtime.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped in this process (" + ", ".join(runtimes) +
                          "): libheom must share the one that owns torch's tensors and streams")
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != 0:
        msg = _lib.heom_last_error().decode() if _lib is not None else ""
        raise HeomError(status, msg)
