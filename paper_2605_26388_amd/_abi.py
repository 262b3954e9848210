"""ctypes mirror of include/dg.h and the loader of libdg.so.

There is no fallback: if the library is missing or fails to load, every entry
point raises.  Argument marshalling only; all computation happens in libdg.
"""

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdg.so")

DG_MAX_SPECIES = 8
DG_MAX_REACTIONS = 8

DG_OK, DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP, DG_ERR_OOM, DG_ERR_NONPHYSICAL, DG_ERR_NEWTON = range(7)
DG_EULER, DG_NAVIER_STOKES, DG_REACTING_EULER, DG_REACTING_2T = range(4)
DG_F64, DG_F32 = range(2)
DG_VOLUME_STANDARD, DG_VOLUME_SPLIT = range(2)
DG_BC_PERIODIC, DG_BC_WALL, DG_BC_INFLOW, DG_BC_OUTFLOW = range(4)

EXPORTS = (
    "dg_create", "dg_destroy", "dg_sizes", "dg_node_coords", "dg_rhs", "dg_rk_stage", "dg_rk_stage_dual",
    "dg_ssprk54_step",
    "dg_source_chem", "dg_rhs_adjoint", "dg_rk_stage_adjoint", "dg_dt_cfl", "dg_integrals",
    "dg_integrals_noalloc", "dg_status_read", "dg_strerror", "dg_last_error",
)


class Mechanism(ctypes.Structure):
    _fields_ = [
        ("nspecies", c_int32), ("nreactions", c_int32),
        ("W", c_double * DG_MAX_SPECIES), ("R", c_double * DG_MAX_SPECIES),
        ("cv", c_double * DG_MAX_SPECIES), ("h0", c_double * DG_MAX_SPECIES),
        ("nu_f", (c_int32 * DG_MAX_SPECIES) * DG_MAX_REACTIONS),
        ("nu_b", (c_int32 * DG_MAX_SPECIES) * DG_MAX_REACTIONS),
        ("A_f", c_double * DG_MAX_REACTIONS), ("beta_f", c_double * DG_MAX_REACTIONS),
        ("theta_f", c_double * DG_MAX_REACTIONS),
        ("A_b", c_double * DG_MAX_REACTIONS), ("beta_b", c_double * DG_MAX_REACTIONS),
        ("theta_b", c_double * DG_MAX_REACTIONS),
        ("third_body", c_int32 * DG_MAX_REACTIONS), ("reversible", c_int32 * DG_MAX_REACTIONS),
        ("eff", (c_double * DG_MAX_SPECIES) * DG_MAX_REACTIONS),
        ("kappa_c", c_double), ("kappa_r", c_double),
    ]


class Vibration(ctypes.Structure):
    _fields_ = [
        ("theta_v", c_double * DG_MAX_SPECIES),
        ("mw_a", (c_double * DG_MAX_SPECIES) * DG_MAX_SPECIES),
        ("mw_b", (c_double * DG_MAX_SPECIES) * DG_MAX_SPECIES),
        ("park_sigma", c_double),
        ("two_temp", c_int32 * DG_MAX_REACTIONS),
    ]


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", c_int32), ("degree", c_int32), ("physics", c_int32), ("precision", c_int32),
        ("batch", c_int32), ("nel", c_int32 * 3), ("lo", c_double * 3), ("hi", c_double * 3),
        ("patch_lo", c_int32 * 2), ("patch_hi", c_int32 * 2),
        ("gamma", c_double), ("mu", c_double), ("prandtl", c_double),
        ("mech", POINTER(Mechanism)),
        ("newton_max_iter", c_int32), ("newton_tol", c_double), ("device", c_int32),
        ("volume", c_int32),
        ("rho_floor", c_double), ("p_floor", c_double),
        ("vib", POINTER(Vibration)),
        ("warp", c_double), ("bc", c_int32 * 6), ("bc_state", c_double * 5),
    ]


class Counters(ctypes.Structure):
    _fields_ = [
        ("nonphysical", c_int32), ("newton_unconverged", c_int32), ("species_clips", c_int32),
        ("newton_iters_max", c_int32), ("first_bad", c_int64), ("floored", c_int32),
    ]


_lib = None


def load():
    """Load libdg.so (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2605_26388_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "dg_create": (c_int32, [POINTER(Desc), POINTER(P)]),
        "dg_destroy": (c_int32, [P]),
        "dg_sizes": (c_int32, [P, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32)]),
        "dg_node_coords": (c_int32, [P, P, P]),
        "dg_rhs": (c_int32, [P, P, P, P]),
        "dg_rk_stage": (c_int32, [P, P, P, P, c_double, c_double, c_double, P]),
        "dg_rk_stage_dual": (c_int32, [P, P, P, P, c_double, c_double, c_double, P, P, c_double, c_double,
                                       c_double, P]),
        "dg_ssprk54_step": (c_int32, [P, P, c_double, P, P, P, P]),
        "dg_source_chem": (c_int32, [P, P, P, c_double, c_int32, P]),
        "dg_rhs_adjoint": (c_int32, [P, P, P, P, P]),
        "dg_rk_stage_adjoint": (c_int32, [P, P, P, P, P, c_double, c_double, c_double, c_int32, P]),
        "dg_dt_cfl": (c_int32, [P, P, c_double, POINTER(c_double), P]),
        "dg_integrals": (c_int32, [P, P, POINTER(c_double), P]),
        "dg_integrals_noalloc": (c_int32, [P, P, P, P]),
        "dg_status_read": (c_int32, [P, POINTER(Counters), c_int32, P]),
        "dg_strerror": (ctypes.c_char_p, [c_int32]),
        "dg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def check(code, what):
    if code != DG_OK:
        lib = load()
        detail = lib.dg_last_error().decode()
        raise DGError(code, f"{what}: {lib.dg_strerror(code).decode()}: {detail}")
