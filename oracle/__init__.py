"""CPU oracle for the batched post-Newtonian inspiral integrator.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this package.  It shares no code with the GPU library and does
not import it.  The arithmetic lives in pn_oracle.cpp (plain FP64 C++);
this module only marshals numpy arrays through ctypes.

All arrays are structure-of-arrays float64 with component c of inspiral i
at [c, i]:  m [2, n], S0 [6, n], L0 [3, n], omega0 [n], y [10, n] with
y = (omega, S1, S2, L_hat).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build as _build

# Term switches (bit values shared with the GPU library's interface).
TERM_PN = 1
TERM_SO_WDOT = 2
TERM_SS_WDOT = 4
TERM_RR = 8
TERM_SO_PREC = 16
TERM_SS_PREC = 32
TERM_ALL = 63

STATUS = {0: "OK", 1: "DONE_AT_START", -1: "MAX_STEPS", -2: "H_UNDERFLOW",
          -3: "NONFINITE", -4: "BAD_INPUT", -5: "OMEGADOT_NONPOSITIVE"}


class _Opts(C.Structure):
    _fields_ = [
        ("h0", C.c_double), ("h_fixed", C.c_double), ("t_end", C.c_double),
        ("max_steps", C.c_int64), ("terms", C.c_int32), ("theta_literal", C.c_int32),
        ("replay", C.c_void_p), ("n_replay_t", C.c_void_p), ("n_replay_w", C.c_void_p),
        ("replay_stride", C.c_int64),
        ("record", C.c_void_p), ("record_stride", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        L = C.CDLL(LIB)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.oracle_rhs.argtypes = [i64, vp, vp, vp, i32, i32]
        L.oracle_integrate.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, C.POINTER(_Opts),
                                       vp, vp, vp, vp, vp, vp, i32]
        L.oracle_tangent.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, dbl, dbl,
                                     C.POINTER(_Opts), vp, vp, vp, vp, vp, i32]
        L.oracle_observables.argtypes = [i64, vp, vp]
        L.oracle_count_ops.argtypes = [vp, vp, dbl, dbl, C.POINTER(_Opts), vp, vp, vp]
        L.oracle_tableau.argtypes = [vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _opts(h0=0.0, h_fixed=0.0, t_end=0.0, max_steps=0, terms=TERM_ALL, theta_literal=0):
    o = _Opts()
    o.h0, o.h_fixed, o.t_end = float(h0), float(h_fixed), float(t_end)
    o.max_steps, o.terms, o.theta_literal = int(max_steps), int(terms), int(theta_literal)
    o.replay = o.n_replay_t = o.n_replay_w = o.record = None
    o.replay_stride = o.record_stride = 0
    return o


def rhs(m, y, terms=TERM_ALL, theta_literal=0):
    """Eqs. (1)-(4) at each state: m [2, n], y [10, n] -> dy/dt [10, n]."""
    y = _f64(y)
    n = y.shape[1]
    m = _f64(m, (2, n))
    out = np.empty((10, n))
    lib().oracle_rhs(n, _p(m), _p(y), _p(out), int(terms), int(theta_literal))
    return out


def integrate(m, S0, L0, omega0, omega_f, tol, *, h0=0.0, h_fixed=0.0, t_end=0.0,
              max_steps=0, terms=TERM_ALL, theta_literal=0, record=0, replay=None,
              phase=False, nthreads=0):
    """Integrate each inspiral from omega0 to omega_f (Sec. II).

    record > 0 keeps up to `record` accepted step sizes per inspiral (for replay).
    replay = dict(h=[n, k], n_t=[n], n_w=[n]) re-runs a recorded step sequence.
    phase=True also integrates the orbital phase (d Phi/dt = omega, Phi(0) = 0).
    Returns dict(y [10, n], t [n], steps [3, n] int64 (accepted, rejected, RHS
    evaluations), status [n], n_tw [2, n], phase [n] when asked for, and
    h_record/n_t/n_w when recording).
    """
    omega0 = _f64(omega0)
    n = omega0.shape[0]
    m = _f64(m, (2, n)); S0 = _f64(S0, (6, n)); L0 = _f64(L0, (3, n))
    o = _opts(h0, h_fixed, t_end, max_steps, terms, theta_literal)
    keep = []
    if record:
        rec = np.full((n, int(record)), np.nan)
        o.record = rec.ctypes.data; o.record_stride = int(record); keep.append(rec)
    if replay is not None:
        rh = _f64(replay["h"]); nt = np.ascontiguousarray(replay["n_t"], dtype=np.int32)
        nw = np.ascontiguousarray(replay["n_w"], dtype=np.int32)
        o.replay = rh.ctypes.data; o.n_replay_t = nt.ctypes.data; o.n_replay_w = nw.ctypes.data
        o.replay_stride = rh.shape[1]; keep += [rh, nt, nw]
    y = np.empty((10, n)); t = np.empty(n); steps = np.empty((3, n), dtype=np.int64)
    status = np.empty(n, dtype=np.int32); ntw = np.empty((2, n), dtype=np.int32)
    ph = np.empty(n) if phase else None
    lib().oracle_integrate(n, _p(m), _p(S0), _p(L0), _p(omega0), float(omega_f), float(tol),
                           C.byref(o), _p(y), _p(t), _p(steps), _p(status), _p(ntw), _p(ph),
                           int(nthreads))
    out = {"y": y, "t": t, "steps": steps, "status": status, "n_tw": ntw}
    if phase:
        out["phase"] = ph
    if record:
        out["h_record"] = keep[0]
        out["replay"] = {"h": keep[0], "n_t": ntw[0].copy(), "n_w": ntw[1].copy()}
    return out


def tangent(m, S0, L0, omega0, dm, dS0, dL0, domega0, omega_f, tol, replay, *,
            terms=TERM_ALL, theta_literal=0, nthreads=0):
    """Forward-mode derivative of the replayed integration along one direction."""
    omega0 = _f64(omega0)
    n = omega0.shape[0]
    m = _f64(m, (2, n)); S0 = _f64(S0, (6, n)); L0 = _f64(L0, (3, n))
    dm = _f64(dm, (2, n)); dS0 = _f64(dS0, (6, n)); dL0 = _f64(dL0, (3, n))
    domega0 = _f64(domega0, (n,))
    o = _opts(terms=terms, theta_literal=theta_literal)
    rh = _f64(replay["h"]); nt = np.ascontiguousarray(replay["n_t"], dtype=np.int32)
    nw = np.ascontiguousarray(replay["n_w"], dtype=np.int32)
    o.replay = rh.ctypes.data; o.n_replay_t = nt.ctypes.data; o.n_replay_w = nw.ctypes.data
    o.replay_stride = rh.shape[1]
    y = np.empty((10, n)); dy = np.empty((10, n)); t = np.empty(n); dt = np.empty(n)
    status = np.empty(n, dtype=np.int32)
    rc = lib().oracle_tangent(n, _p(m), _p(S0), _p(L0), _p(omega0), _p(dm), _p(dS0), _p(dL0),
                              _p(domega0), float(omega_f), float(tol), C.byref(o), _p(y),
                              _p(dy), _p(t), _p(dt), _p(status), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_tangent failed")
    return {"y": y, "dy": dy, "t": t, "dt": dt, "status": status}


def observables(y):
    """(S1_hat.S2_hat, S1_hat.L_hat, S2_hat.L_hat) of each state: [10, n] -> [3, n]."""
    y = _f64(y)
    n = y.shape[1]
    out = np.empty((3, n))
    lib().oracle_observables(n, _p(y), _p(out))
    return out


def count_ops(m, y0, omega_f, tol, **kw):
    """Operation counts of one RHS evaluation and of one whole adaptive run.

    Returns dict(rhs=..., run=..., accepted, rejected, nrhs) with each count a
    dict over add, mul, div, cbrt, log, sqrt, pow (state-dependent ops only).
    """
    m = _f64(m, (2,)); y0 = _f64(y0, (10,))
    o = _opts(**kw)
    cr = np.zeros(7, dtype=np.int64); cu = np.zeros(7, dtype=np.int64)
    info = np.zeros(3, dtype=np.int64)
    st = lib().oracle_count_ops(_p(m), _p(y0), float(omega_f), float(tol), C.byref(o),
                                _p(cr), _p(cu), _p(info))
    keys = ("add", "mul", "div", "cbrt", "log", "sqrt", "pow")
    return {"rhs": dict(zip(keys, cr.tolist())), "run": dict(zip(keys, cu.tolist())),
            "accepted": int(info[0]), "rejected": int(info[1]), "nrhs": int(info[2]),
            "status": int(st)}


def tableau():
    """The Dormand-Prince tableau as exact (numerator, denominator) pairs."""
    a = np.zeros((7, 6, 2)); b = np.zeros((7, 2)); bh = np.zeros((7, 2)); c = np.zeros((7, 2))
    lib().oracle_tableau(_p(a), _p(b), _p(bh), _p(c))
    return a, b, bh, c
