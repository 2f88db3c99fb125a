"""ctypes declarations of the C ABI in include/sdc.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdc.so")

MAX_NODES = 6
MAX_SWEEPS = 16
MAX_RECORDINGS = 64
NOALLOC_MAX_IN = 1 << 24

SDC_OK = 0
ERRORS = {
    -1: "SDC_ERR_ARG", -2: "SDC_ERR_HIP", -3: "SDC_ERR_CG_MAXIT", -4: "SDC_ERR_STATE",
    -5: "SDC_ERR_OOM", -6: "SDC_ERR_NONFINITE",
}


class Params(ctypes.Structure):
    _fields_ = [("M", c_int32), ("K", c_int32), ("dt", c_double), ("theta", c_double),
                ("cg_rtol", c_double), ("cg_maxit", c_int32), ("format", c_int32),
                ("K_min", c_int32), ("tol_sdc", c_double), ("rho", c_double), ("drop_mode", c_int32),
                ("scheme", c_int32), ("first_rings", c_int32), ("first_full_every", c_int32),
                ("small_set_rows", c_int32), ("rows_per_thread", c_int32), ("cg_energy_tol", c_double),
                ("cg_delay", c_int32)]


class SweepStats(ctypes.Structure):
    _fields_ = [("n_active", c_int64), ("nnz_active", c_int64), ("n_next", c_int64),
                ("cg_iters_max", c_int32 * MAX_NODES), ("cg_row_iters", c_int64 * MAX_NODES),
                ("cg_nnz_iters", c_int64 * MAX_NODES), ("energy", c_double), ("n_stopped", c_int32),
                ("ms", c_double)]

    def as_dict(self, M):
        return {
            "n_active": self.n_active, "nnz_active": self.nnz_active, "n_next": self.n_next,
            "cg_iters_max": list(self.cg_iters_max[:M]),
            "cg_row_iters": list(self.cg_row_iters[:M]),
            "cg_nnz_iters": list(self.cg_nnz_iters[:M]),
            "energy": self.energy, "n_stopped": self.n_stopped, "ms": self.ms,
        }


class StepStats(ctypes.Structure):
    _fields_ = [("n_sweeps", c_int32), ("sweep", SweepStats * MAX_SWEEPS)]


class ProfileStats(ctypes.Structure):
    _fields_ = [("cg_launches", c_int64), ("cg_ms", c_double), ("cg_bytes", c_double),
                ("cg_all_launches", c_int64), ("cg_all_ms", c_double), ("cg_all_bytes", c_double),
                ("cg_rows", c_double), ("cg_nnz", c_double), ("cg_all_rows", c_double), ("cg_all_nnz", c_double)]


class Info(ctypes.Structure):
    _fields_ = [("format", c_int32), ("n_diagonals", c_int32), ("t_csr_us", c_double),
                ("t_dia_us", c_double), ("redone_steps", c_int64), ("rows_per_thread", c_int32),
                ("t_rows1_us", c_double), ("t_rows2_us", c_double), ("graph_steps", c_int64),
                ("graph_captures", c_int64), ("graph_redone", c_int64), ("t_sell_us", c_double),
                ("xcd_chunk", c_int32)]


class Emi(ctypes.Structure):
    """sdc_emi: cell-by-cell couplings (host arrays, copied by the setup)."""
    _fields_ = [("n_mem", c_int64), ("mem_intra", c_void_p), ("mem_extra", c_void_p), ("mem_len", c_void_p),
                ("cm", c_double), ("n_gap", c_int64), ("gap_a", c_void_p), ("gap_b", c_void_p),
                ("gap_len", c_void_p), ("g_gap", c_double), ("robin_len", c_void_p), ("eps", c_double)]


PTR = c_void_p
P_I64 = POINTER(c_int64)
P_I32 = POINTER(c_int32)

SIGNATURES = {
    "sdc_create": (c_int32, [POINTER(c_void_p), c_int32, c_void_p]),
    "sdc_destroy": (None, [c_void_p]),
    "sdc_last_error": (c_char_p, [c_void_p]),
    "sdc_set_stream": (c_int32, [c_void_p, c_void_p]),
    "sdc_setup_mesh": (c_int32, [c_void_p, POINTER(Params), c_int32, c_int32, PTR, PTR, PTR, PTR,
                                 PTR, PTR, PTR, POINTER(Emi)]),
    "sdc_add_stimulus": (c_int32, [c_void_p, c_double, PTR, c_int64, c_double]),
    "sdc_get_sizes": (c_int32, [c_void_p, P_I64, P_I64, P_I64]),
    "sdc_get_system": (c_int32, [c_void_p, PTR, PTR, PTR, PTR]),
    "sdc_step": (c_int32, [c_void_p, PTR, PTR, c_double, POINTER(StepStats)]),
    "sdc_begin_step": (c_int32, [c_void_p, PTR, PTR, c_double]),
    "sdc_sweep": (c_int32, [c_void_p, POINTER(SweepStats)]),
    "sdc_end_step": (c_int32, [c_void_p, PTR, PTR]),
    "sdc_get_node": (c_int32, [c_void_p, c_int32, PTR, PTR]),
    "sdc_get_active": (c_int32, [c_void_p, PTR, P_I64]),
    "sdc_get_cg_iters": (c_int32, [c_void_p, PTR]),
    "sdc_set_active": (c_int32, [c_void_p, c_int32, PTR, c_int64]),
    "sdc_solve": (c_int32, [c_void_p, c_int32, PTR, c_int64, PTR, PTR, P_I32]),
    "sdc_select": (c_int32, [c_void_p, PTR, PTR, c_int64, c_double, PTR, P_I64]),
    "sdc_collocation": (c_int32, [c_int32, PTR, PTR, PTR, PTR]),
    "sdc_profile": (c_int32, [c_void_p, c_int32]),
    "sdc_set_graph": (c_int32, [c_void_p, c_int32]),
    "sdc_get_info": (c_int32, [c_void_p, POINTER(Info)]),
    "sdc_get_drop_tolerance": (c_int32, [c_void_p, PTR]),
    "sdc_adjoint_step": (c_int32, [c_void_p, PTR, PTR, c_double, PTR, PTR, PTR, PTR]),
    "sdc_set_coefficients": (c_int32, [c_void_p, PTR, PTR]),
    "sdc_adjoint_record": (c_int32, [c_void_p, c_int32, PTR, PTR, c_double]),
    "sdc_adjoint_reverse": (c_int32, [c_void_p, c_int32, PTR, PTR, PTR, PTR]),
    "sdc_profile_read": (c_int32, [c_void_p, POINTER(ProfileStats)]),
    "sdc_select_noalloc": (c_int32, [c_int32, c_void_p, PTR, c_int64, PTR, c_int64, c_double, PTR, PTR]),
}

_lib = None


def load():
    """Load libsdc.so (once) and declare every ABI function."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run python -m paper_2311_07206_amd.build "
                           "(or python paper_2311_07206_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
