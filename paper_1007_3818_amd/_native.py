"""ctypes view of libgamer_hydro.so (the C ABI in include/gamer_hydro.h).

Argument marshalling only.  Loading fails loudly when the library has not been
built; there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgamer_hydro.so")

GAMER_OK = 0
GAMER_EINVAL = -1
GAMER_EHIP = -2
GAMER_ENOMEM = -3
MAX_LEVELS = 32
NOALLOC_MAX_GROUPS = 262144

_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64


LIMIT_PRIMITIVE = 0
LIMIT_CHARACTERISTIC = 1


class GamerOpts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("variant", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("limiting", ctypes.c_int32), ("zseg", ctypes.c_int32),
                ("bad_count_dev", ctypes.c_void_p)]


_PO = ctypes.POINTER(GamerOpts)

# name -> (restype, argtypes), in the order of include/gamer_hydro.h
SIGNATURES = {
    "gamer_version": (_I, []),
    "gamer_set_stream": (_I, [_P]),
    "gamer_get_stream": (_P, []),
    "gamer_last_error": (ctypes.c_char_p, []),
    "gamer_solver_variants": (_I, [_I]),
    "gamer_solver_variant_shape": (_I, [_I, _I, _P, _P]),
    "gamer_hydro_solve": (_I, [_P, _I64, _D, _D, _D, _P, _P]),
    "gamer_hydro_solve_f32": (_I, [_P, _I64, _D, _D, _D, _P, _P]),
    "gamer_hydro_solve_batched": (_I, [_P, _I64, _P, _P, _P, _I, _D, _P, _P, _P, _PO, _P]),
    "gamer_hydro_solve_batched_f32": (_I, [_P, _I64, _P, _P, _P, _I, _D, _P, _P, _P, _PO, _P]),
    "gamer_hydro_solve_periodic": (_I, [_P, _I, _I, _I, _P, _P, _D, _P, _P, _P, _PO]),
    "gamer_hydro_solve_periodic_f32": (_I, [_P, _I, _I, _I, _P, _P, _D, _P, _P, _P, _PO]),
    "gamer_hydro_solve_batched_mixed": (_I, [_P, _I64, _P, _P, _P, _I, _D, _P, _P, _P, _PO, _P]),
    "gamer_hydro_solve_periodic_mixed": (_I, [_P, _I, _I, _I, _P, _P, _D, _P, _P, _P, _PO]),
    "gamer_step_reduce": (_I, [_P, _I64, _P, _P, _I, _D, _P, _P]),
    "gamer_group_stats": (_I, [_P, _I64, _D, _P]),
    "gamer_group_stats_f32": (_I, [_P, _I64, _D, _P]),
    "gamer_cfl_dt": (_I, [_P, _I64, _D, _D, _D, _P, _I]),
    "gamer_cfl_dt_f32": (_I, [_P, _I64, _D, _D, _D, _P, _I]),
    "gamer_cfl_dt_noalloc": (_I, [_P, _I64, _D, _D, _D, _P]),
    "gamer_conserved_sums": (_I, [_P, _I64, _D, _P, _I]),
    "gamer_conserved_sums_f32": (_I, [_P, _I64, _D, _P, _I]),
    "gamer_pack_periodic": (_I, [_P, _I, _I, _I, _P]),
    "gamer_pack_periodic_f32": (_I, [_P, _I, _I, _I, _P]),
    "gamer_ctu_workspace_bytes": (ctypes.c_size_t, [_I64, _I]),
    "gamer_ctu_solve_batched": (_I, [_P, _I64, _P, _P, _P, _I, _D, _P, _P, _P, _PO, _P, ctypes.c_size_t]),
    "gamer_ctu_solve_batched_f32": (_I, [_P, _I64, _P, _P, _P, _I, _D, _P, _P, _P, _PO, _P,
                                         ctypes.c_size_t]),
    "gamer_rtvd_workspace_bytes": (ctypes.c_size_t, [_I64, _I]),
    "gamer_rtvd_solve_batched": (_I, [_P, _I64, _P, _P, _P, _I, _D, _I, _P, ctypes.c_size_t, _P]),
    "gamer_rtvd_solve_batched_f32": (_I, [_P, _I64, _P, _P, _P, _I, _D, _I, _P, ctypes.c_size_t, _P]),
    "gamer_rtvd_solve_periodic": (_I, [_P, _I, _I, _I, _P, _P, _D, _I, _P, ctypes.c_size_t, _P]),
    "gamer_rtvd_solve_periodic_f32": (_I, [_P, _I, _I, _I, _P, _P, _D, _I, _P, ctypes.c_size_t, _P]),
    "gamer_flux_accumulate": (_I, [_P, _I64, _P, _I, _P]),
    "gamer_flux_accumulate_f32": (_I, [_P, _I64, _P, _I, _P]),
    "gamer_flux_correct": (_I, [_P, _I64, _P, _P, _I64, _P, _I64, _P, _P, _P]),
    "gamer_flux_correct_f32": (_I, [_P, _I64, _P, _P, _I64, _P, _I64, _P, _P, _P]),
    "gamer_restrict": (_I, [_P, _P, _I64, _P, _I64, _P]),
    "gamer_restrict_f32": (_I, [_P, _P, _I64, _P, _I64, _P]),
}

_lib = None


class GamerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gamer error {code}: {msg}")
        self.code = code


def lib():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_1007_3818_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != GAMER_OK:
        msg = lib().gamer_last_error()
        raise GamerError(rc, msg.decode() if msg else "")
    return rc
