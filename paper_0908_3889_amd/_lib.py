"""ctypes declarations of the C interface in include/pn.h (argument
marshalling only).  Loading fails loudly when libpn.so has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PN_LIB may name another build of the same library (for A/B timing)
LIB_PATH = os.environ.get("PN_LIB") or os.path.join(HERE, "libpn.so")

# return codes
PN_OK, PN_EINVAL, PN_ENODEV, PN_EHIP, PN_ENOMEM, PN_EBUSY = 0, -1, -2, -3, -4, -5
# per-inspiral status
STATUS = {0: "OK", 1: "DONE_AT_START", -1: "MAX_STEPS", -2: "H_UNDERFLOW", -3: "NONFINITE",
          -4: "BAD_INPUT", -5: "OMEGADOT_NONPOSITIVE", -6: "TAPE_FULL"}
PN_ST_TAPE_FULL = -6
# term switches
PN_TERM_PN, PN_TERM_SO_WDOT, PN_TERM_SS_WDOT, PN_TERM_RR = 1, 2, 4, 8
PN_TERM_SO_PREC, PN_TERM_SS_PREC, PN_TERM_ALL = 16, 32, 63
# schedules and arithmetic
PN_SCHED_PERSISTENT, PN_SCHED_STATIC = 0, 1
PN_PREC_FP64, PN_PREC_FP32_SPLIT, PN_PREC_FP32_STATE = 0, 1, 2

EXPORTS = ("pn_integrate", "pn_rhs", "pn_observables", "pn_strerror", "pn_version",
           "pn_tape_stride", "pn_integrate_record", "pn_adjoint_workspace_bytes",
           "pn_integrate_adjoint", "pn_histogram", "pn_histogram2d", "pn_pearson", "pn_kde",
           "pn_ks_workspace_bytes", "pn_ks_uniform", "pn_stats_workspace_bytes", "pn_generate",
           "pn_autotune", "pn_integrate_phase", "pn_fma_rate", "pn_shutdown", "pn_integrate_noalloc", "pn_cost_order", "pn_cost_order_workspace_bytes",
           "pn_check_integrate_host", "pn_check_start", "pn_check_finish", "pn_ckpt_bytes",
           "pn_integrate_replay", "pn_fma_lanes")


class PnOpts(C.Structure):
    _fields_ = [
        ("h0", C.c_double),
        ("h_fixed", C.c_double),
        ("t_end", C.c_double),
        ("max_steps", C.c_int64),
        ("terms", C.c_int32),
        ("theta_literal", C.c_int32),
        ("schedule", C.c_int32),
        ("block", C.c_int32),
        ("waves_per_simd", C.c_int32),
        ("refill_min", C.c_int32),
        ("precision", C.c_int32),
        ("order", C.c_void_p),
        ("packed", C.c_void_p),
    ]


class PnGenSpec(C.Structure):
    _fields_ = [("q_lo", C.c_double), ("q_hi", C.c_double), ("chi1_lo", C.c_double), ("chi1_hi", C.c_double),
                ("chi2_lo", C.c_double), ("chi2_hi", C.c_double), ("omega0_lo", C.c_double),
                ("omega0_hi", C.c_double), ("seed", C.c_uint64)]


class PnCheckReport(C.Structure):
    _fields_ = [("checked", C.c_int64), ("status_mismatches", C.c_int64), ("step_mismatches", C.c_int64),
                ("flagged", C.c_int64), ("max_dot_diff", C.c_double), ("host_seconds", C.c_double)]


class PnError(RuntimeError):
    pass


_lib = None


def load():
    """The loaded libpn.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PnError(f"{LIB_PATH} is not built; run `python -m paper_0908_3889_amd.build` "
                      "(the GPU path has no fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
    popts = C.POINTER(PnOpts)
    L.pn_integrate.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, vp, vp, vp, vp, vp, vp]
    L.pn_integrate.restype = C.c_int
    L.pn_cost_order_workspace_bytes.argtypes = [i64]
    L.pn_cost_order_workspace_bytes.restype = C.c_size_t
    L.pn_cost_order.argtypes = [i64, i64, vp, vp, vp, vp, dbl, vp, vp, C.c_size_t, vp, vp]
    L.pn_cost_order.restype = C.c_int
    L.pn_check_integrate_host.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, vp, vp, vp, vp, C.c_int32]
    L.pn_check_integrate_host.restype = C.c_int
    L.pn_check_start.argtypes = [C.POINTER(vp), i64, i64, vp, vp, vp, vp, dbl, dbl, popts, C.c_int32]
    L.pn_check_start.restype = C.c_int
    L.pn_check_finish.argtypes = [vp, vp, vp, vp, i64, dbl, vp, C.POINTER(PnCheckReport)]
    L.pn_check_finish.restype = C.c_int
    L.pn_integrate_noalloc.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, vp, vp, vp, vp, vp, vp]
    L.pn_integrate_noalloc.restype = C.c_int
    L.pn_integrate_phase.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, vp, vp, vp, vp, vp, vp, vp]
    L.pn_integrate_phase.restype = C.c_int
    L.pn_fma_rate.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    L.pn_fma_rate.restype = C.c_int
    L.pn_shutdown.argtypes = []
    L.pn_shutdown.restype = C.c_int
    L.pn_rhs.argtypes = [i64, i64, vp, vp, vp, popts, vp]
    L.pn_rhs.restype = C.c_int
    L.pn_observables.argtypes = [i64, i64, vp, vp, vp]
    L.pn_observables.restype = C.c_int
    L.pn_strerror.argtypes = [C.c_int]
    L.pn_strerror.restype = C.c_char_p
    L.pn_version.argtypes = []
    L.pn_version.restype = C.c_char_p
    L.pn_tape_stride.argtypes = [i64, C.c_int32]
    L.pn_tape_stride.restype = C.c_size_t
    L.pn_integrate_record.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, vp, vp, vp, vp, vp,
                                      vp, i64, C.c_int32, vp]
    L.pn_integrate_record.restype = C.c_int
    L.pn_adjoint_workspace_bytes.argtypes = [i64, C.c_int32]
    L.pn_adjoint_workspace_bytes.restype = C.c_size_t
    L.pn_integrate_adjoint.argtypes = [i64, i64, vp, dbl, popts, vp, i64, C.c_int32, vp, vp, vp, vp, vp,
                                       vp, vp, vp, C.c_size_t, vp, vp]
    L.pn_integrate_adjoint.restype = C.c_int
    L.pn_fma_lanes.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    L.pn_fma_lanes.restype = C.c_int
    L.pn_ckpt_bytes.argtypes = [i64, i64, C.c_int32]
    L.pn_ckpt_bytes.restype = C.c_size_t
    L.pn_integrate_replay.argtypes = [i64, i64, vp, vp, vp, vp, dbl, popts, vp, i64, C.c_int32, vp, vp, vp, vp]
    L.pn_integrate_replay.restype = C.c_int
    i32, sz = C.c_int32, C.c_size_t
    L.pn_histogram.argtypes = [i64, i64, vp, i32, i32, dbl, dbl, vp, vp]
    L.pn_histogram.restype = C.c_int
    L.pn_histogram2d.argtypes = [i64, i64, vp, vp, i32, i32, dbl, dbl, vp, vp]
    L.pn_histogram2d.restype = C.c_int
    L.pn_pearson.argtypes = [i64, i64, vp, vp, i32, vp, vp, sz, vp]
    L.pn_pearson.restype = C.c_int
    L.pn_kde.argtypes = [i64, i64, vp, i32, vp, i64, i32, dbl, dbl, vp, vp, sz, vp]
    L.pn_kde.restype = C.c_int
    L.pn_ks_workspace_bytes.argtypes = [i64]
    L.pn_ks_workspace_bytes.restype = sz
    L.pn_ks_uniform.argtypes = [i64, i64, vp, i32, dbl, dbl, vp, vp, sz, vp]
    L.pn_ks_uniform.restype = C.c_int
    L.pn_stats_workspace_bytes.argtypes = [i64, i32, i32]
    L.pn_stats_workspace_bytes.restype = sz
    L.pn_autotune.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, popts, i64, i32, vp, vp, vp, vp, vp, popts,
                              vp, vp]
    L.pn_autotune.restype = C.c_int
    L.pn_generate.argtypes = [i64, i64, i64, C.POINTER(PnGenSpec), vp, vp, vp, vp, vp]
    L.pn_generate.restype = C.c_int
    _lib = L
    return L


def check(rc: int, what: str) -> None:
    if rc != PN_OK:
        msg = load().pn_strerror(rc).decode()
        raise PnError(f"{what} failed: {msg} ({rc})")
