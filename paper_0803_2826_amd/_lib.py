"""ctypes binding of liblbmi.so: the C ABI of include/lb.h with the same names.

Argument marshalling only.  Every numerical step runs in the HIP kernels of
the library; if the library is missing or fails to load this module raises,
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmi.so")

LB_OK = 0
LB_EINVAL = -1
LB_ENOMEM = -2
LB_EDEVICE = -3
LB_ENONFINITE = -4
LB_ESTATE = -5
LB_EUNSUPPORTED = -6
LB_EIO = -7

LB_F64, LB_F32, LB_BF16, LB_F16 = 0, 1, 2, 3

STATUS_NAMES = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EDEVICE", -4: "LB_ENONFINITE",
                -5: "LB_ESTATE", -6: "LB_EUNSUPPORTED", -7: "LB_EIO"}

# Every symbol declared in include/lb.h.
EXPORTS = (
    "lb_create", "lb_destroy", "lb_init_equilibrium", "lb_set_populations", "lb_get_populations", "lb_step",
    "lb_couple", "lb_coupled_steps", "lb_moments", "lb_totals", "lb_totals_exact", "lb_negative_count", "lb_mode_stats", "lb_noise_sample", "lb_sync", "lb_step_count",
    "lb_set_step_count", "lb_last_error", "lb_create_batch", "lb_vacf", "lb_launch_config", "lb_save", "lb_load", "lb_backward_coupled",
    "lb_tape_begin", "lb_tape_reserve", "lb_backward", "lb_step_noalloc", "lb_params_two_rate",
)


LB_ROUND_NEAREST, LB_ROUND_STOCHASTIC = 0, 1
LB_BOND_HARMONIC, LB_BOND_FENE = 0, 1
LB_NOISE_GAUSSIAN, LB_NOISE_THREE_POINT = 0, 1


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("rho0", ctypes.c_double),
        ("gamma_shear", ctypes.c_double), ("gamma_bulk", ctypes.c_double),
        ("gamma_3a", ctypes.c_double), ("gamma_3b", ctypes.c_double),
        ("gamma_4a", ctypes.c_double), ("gamma_4b", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64),
        ("noise_rho0", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("track_totals", ctypes.c_int32),
        ("box_id", ctypes.c_int32),
        ("vacf_lags", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
        ("rounding", ctypes.c_int32),
        ("walls", ctypes.c_int32),
    ]


class lb_beads(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("nbonds", ctypes.c_int32),
        ("pos", ctypes.c_void_p), ("mom", ctypes.c_void_p),
        ("mass", ctypes.c_void_p), ("zeta", ctypes.c_void_p),
        ("bonds", ctypes.c_void_p),
        ("k_bond", ctypes.c_double), ("r0", ctypes.c_double),
        ("fext", ctypes.c_void_p),
        ("stencil", ctypes.c_int32), ("bond", ctypes.c_int32),
        ("wca_epsilon", ctypes.c_double), ("wca_sigma", ctypes.c_double),
        ("noise", ctypes.c_int32),
    ]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load liblbmi.so (importing torch first so both share one HIP runtime).
    LBMI_LIBRARY may name another build of the same library."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("LBMI_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"liblbmi.so not built at {path}; run python -m paper_0803_2826_amd.build")
    import torch  # noqa: F401  (loads the HIP runtime the library will share)
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.lb_create.argtypes = [ctypes.POINTER(lb_params), vp, ctypes.POINTER(vp)]
    L.lb_destroy.argtypes = [vp]
    L.lb_init_equilibrium.argtypes = [vp, vp, vp]
    L.lb_set_populations.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32]
    L.lb_get_populations.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32]
    L.lb_step.argtypes = [vp, ctypes.c_int32]
    L.lb_couple.argtypes = [vp, ctypes.POINTER(lb_beads)]
    L.lb_coupled_steps.argtypes = [vp, ctypes.POINTER(lb_beads), ctypes.c_int32]
    L.lb_moments.argtypes = [vp, vp, vp]
    L.lb_totals.argtypes = [vp, dp]
    L.lb_totals_exact.argtypes = [vp, dp]
    L.lb_negative_count.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), dp]
    L.lb_mode_stats.argtypes = [vp, dp]
    L.lb_noise_sample.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, vp]
    L.lb_sync.argtypes = [vp]
    L.lb_step_count.argtypes = [vp]
    L.lb_step_count.restype = ctypes.c_uint64
    L.lb_set_step_count.argtypes = [vp, ctypes.c_uint64]
    L.lb_create_batch.argtypes = [ctypes.POINTER(lb_params), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp,
                                  ctypes.POINTER(vp)]
    L.lb_vacf.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
    L.lb_launch_config.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.lb_tape_begin.argtypes = [vp, ctypes.c_int32]
    L.lb_tape_reserve.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(lb_beads)]
    L.lb_backward.argtypes = [vp, vp, ctypes.c_int32, vp, dp]
    L.lb_backward_coupled.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp, dp, vp, vp]
    L.lb_save.argtypes = [vp, ctypes.c_char_p]
    L.lb_load.argtypes = [vp, ctypes.c_char_p]
    L.lb_step_noalloc.argtypes = [ctypes.POINTER(lb_params), vp, vp, ctypes.c_uint64, vp, vp]
    L.lb_params_two_rate.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.POINTER(lb_params)]
    L.lb_last_error.argtypes = [vp]
    L.lb_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lb_step_count", "lb_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int, ctx=None) -> None:
    if rc != LB_OK:
        L = load()
        msg = L.lb_last_error(ctx).decode() if L is not None else ""
        raise LBError(rc, msg)
