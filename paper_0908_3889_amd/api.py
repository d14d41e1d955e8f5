"""Python binding of the gfx950 integrator.

Same names as the C interface (include/pn.h).  Arguments are torch tensors
on the current HIP device (float64, structure-of-arrays [components, n],
unit stride along n); the functions only marshal pointers, sizes and the
current stream into the library.  Every step of the integration runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

import torch

from . import _lib
from ._lib import PnOpts, check, load

SCHEDULES = {"persistent": _lib.PN_SCHED_PERSISTENT, "static": _lib.PN_SCHED_STATIC}
PRECISIONS = {"fp64": _lib.PN_PREC_FP64, "fp32split": _lib.PN_PREC_FP32_SPLIT, "fp32": _lib.PN_PREC_FP32_STATE}


def _on_current_device(t: torch.Tensor, name: str) -> None:
    # the library works on the current HIP device
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}, but the current device is "
                         f"cuda:{torch.cuda.current_device()} (use torch.cuda.set_device)")


def _soa(t: torch.Tensor, comps: int, n: int, name: str, dtype=torch.float64) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    _on_current_device(t, name)
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if comps == 1:
        if t.dim() != 1 or t.shape[0] != n or (n > 1 and t.stride(0) != 1):
            raise ValueError(f"{name} must have shape [{n}] with unit stride")
    else:
        if t.dim() != 2 or t.shape[0] != comps or t.shape[1] != n or (n > 1 and t.stride(1) != 1):
            raise ValueError(f"{name} must have shape [{comps}, {n}] with unit stride along n")
    return t


def _ld(t: torch.Tensor, n: int) -> int:
    return t.stride(0) if t.dim() == 2 else n


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_opts(*, h0=0.0, h_fixed=0.0, t_end=0.0, max_steps=0, terms=_lib.PN_TERM_ALL,
              theta_literal=0, schedule="persistent", block=0, waves_per_simd=0,
              refill_min=0, precision="fp64", order=None, packed=None) -> PnOpts:
    """pn_opts; order: None or an int32 device tensor [n] (pn_cost_order);
    packed: None or the float64 [n, 16] input records pn_cost_order wrote;
    both kept alive by the returned struct."""
    o = PnOpts()
    o.h0, o.h_fixed, o.t_end = float(h0), float(h_fixed), float(t_end)
    o.max_steps, o.terms, o.theta_literal = int(max_steps), int(terms), int(theta_literal)
    o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.block, o.waves_per_simd, o.refill_min = int(block), int(waves_per_simd), int(refill_min)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    set_order(o, order)
    set_packed(o, packed)
    return o


def set_packed(o: PnOpts, packed) -> PnOpts:
    """Point o.packed at float64 [n, 16] input records (or clear it with None)."""
    if packed is None:
        o.packed = None
        o._packed_ref = None
        return o
    if packed.dtype != torch.float64 or packed.dim() != 2 or packed.shape[1] != 16 or not packed.is_contiguous():
        raise ValueError("packed must be a contiguous float64 [n, 16] tensor")
    o.packed = C.c_void_p(packed.data_ptr())
    o._packed_ref = packed
    return o


def packed_inputs(n: int, device=None):
    """A device buffer for the 128-byte input records of pn_cost_order."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    return torch.empty((int(n), 16), dtype=torch.float64, device=dev)


def set_order(o: PnOpts, order) -> PnOpts:
    """Point o.order at an int32 device tensor (or clear it with None)."""
    if order is None:
        o.order = None
        o._order_ref = None
        return o
    if order.dtype != torch.int32 or order.dim() != 1 or not order.is_contiguous():
        raise ValueError("order must be a contiguous 1-d int32 tensor")
    o.order = C.c_void_p(order.data_ptr())
    o._order_ref = order
    return o


def cost_order_workspace(n: int, device=None):
    """A device workspace tensor for pn_cost_order on n inspirals."""
    b = int(load().pn_cost_order_workspace_bytes(int(n)))
    dev = device or torch.device("cuda", torch.cuda.current_device())
    return torch.empty((max(b, 1),), dtype=torch.uint8, device=dev)


def pn_cost_order(m, S0, L0, omega0, omega_f, out=None, workspace=None, packed=None, stream=None):
    """The longest-first hand-out order of the inspirals (int32 [n] on the
    device) from the leading-order step estimate of pn_cost_order; with
    packed (a float64 [n, 16] buffer, see packed_inputs) the same pass also
    writes the inputs as the records of pn_opts.packed."""
    n = int(omega0.shape[0])
    _soa(omega0, 1, n, "omega0")
    _soa(m, 2, n, "m"); _soa(S0, 6, n, "S0"); _soa(L0, 3, n, "L0")
    lds = {_ld(m, n), _ld(S0, n), _ld(L0, n)}
    if n > 0 and len(lds) != 1:
        raise ValueError("all [components, n] arrays must share one leading dimension")
    ld = lds.pop() if n > 0 else 0
    if out is None:
        out = torch.empty((n,), dtype=torch.int32, device=omega0.device)
    if workspace is None:
        workspace = cost_order_workspace(n, omega0.device)
    if packed is not None and (packed.dtype != torch.float64 or tuple(packed.shape) != (n, 16)
                               or not packed.is_contiguous()):
        raise ValueError("packed must be a contiguous float64 [n, 16] tensor")
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = load().pn_cost_order(n, ld, p(m), p(S0), p(L0), p(omega0), float(omega_f), p(out), p(workspace),
                              int(workspace.numel()), None if packed is None else p(packed), _stream(stream))
    check(rc, "pn_cost_order")
    return out


def alloc_outputs(n: int, device=None, dots: bool = True) -> dict:
    dev = device or torch.device("cuda", torch.cuda.current_device())
    return {
        "y": torch.empty((10, n), dtype=torch.float64, device=dev),
        "t": torch.empty((n,), dtype=torch.float64, device=dev),
        "steps": torch.empty((3, n), dtype=torch.int32, device=dev),
        "status": torch.empty((n,), dtype=torch.int32, device=dev),
        "dots": torch.empty((3, n), dtype=torch.float64, device=dev) if dots else None,
    }


def pn_integrate(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, out=None,
                 dots: bool = True, stream=None) -> dict:
    """Integrate every inspiral from omega0 to omega_f (or to opts.t_end).

    m [2, n], S0 [6, n], L0 [3, n], omega0 [n] (float64, on the GPU).
    Returns dict(y [10, n], t [n], steps [3, n] int32, status [n] int32,
    dots [3, n] or None).  Asynchronous on the current stream.
    """
    return _integrate("plain", m, S0, L0, omega0, omega_f, tol, opts, out, dots, stream)


def _host_soa(a, comps, n, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != ((comps, n) if comps > 1 else (n,)):
        raise ValueError(f"{name}: expected shape {(comps, n) if comps > 1 else (n,)}, got {a.shape}")
    return a


def check_integrate_host(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, nthreads: int = 0) -> dict:
    """The host integrator of the CPU check (pn_check_integrate_host) on
    numpy arrays: dict(y [10, n], t [n], steps [3, n], status [n])."""
    omega0 = np.ascontiguousarray(omega0, dtype=np.float64)
    n = omega0.shape[0]
    m, S0, L0 = _host_soa(m, 2, n, "m"), _host_soa(S0, 6, n, "S0"), _host_soa(L0, 3, n, "L0")
    y = np.empty((10, n)); t = np.empty(n)
    steps = np.empty((3, n), dtype=np.int32); status = np.empty(n, dtype=np.int32)
    o = opts if opts is not None else make_opts()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = load().pn_check_integrate_host(n, n, p(m), p(S0), p(L0), p(omega0), float(omega_f), float(tol),
                                        C.byref(o), p(y), p(t), p(steps), p(status), int(nthreads))
    check(rc, "pn_check_integrate_host")
    return {"y": y, "t": t, "steps": steps, "status": status}


def integrate_checked(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, out=None,
                      fraction: float = 0.01, sample=None, seed: int = 0, dot_tol: float | None = None,
                      nthreads: int = 0, host_inputs: dict | None = None, stream=None):
    """pn_integrate with the CPU check of Sec. III running alongside: a
    random `fraction` of the inspirals (or the indices in `sample`) is
    integrated on host threads (pn_check_start) while the GPU integrates all
    of them, then the GPU's outputs for the sample are compared
    (pn_check_finish).  dot_tol: 1e-8 for FP64, 1e-3 for the FP32 modes
    unless given.  host_inputs: optional numpy copies of the inputs (dict
    m, S, L, omega0), saving the device-to-host copy of the sample.
    Returns (outputs, report dict with the sample indices and their flags)."""
    n = int(omega0.shape[0])
    o = opts if opts is not None else make_opts()
    if sample is None:
        k = max(1, int(round(n * fraction))) if n > 0 else 0
        sample = np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False)) if k else np.zeros(0, np.int64)
    sample = np.asarray(sample, dtype=np.int64)
    k = sample.size
    if k and (sample.min() < 0 or sample.max() >= n):
        raise ValueError("sample indices must lie in [0, n)")
    if host_inputs is not None:
        hm = np.ascontiguousarray(host_inputs["m"][:, sample]); hS = np.ascontiguousarray(host_inputs["S"][:, sample])
        hL = np.ascontiguousarray(host_inputs["L"][:, sample]); hw = np.ascontiguousarray(host_inputs["omega0"][sample])
    else:
        idx = torch.from_numpy(sample).to(omega0.device)
        hm = m[:, idx].cpu().numpy(); hS = S0[:, idx].cpu().numpy()
        hL = L0[:, idx].cpu().numpy(); hw = omega0[idx].cpu().numpy()
    hm, hS, hL, hw = (np.ascontiguousarray(a, dtype=np.float64) for a in (hm, hS, hL, hw))
    handle = C.c_void_p()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = load().pn_check_start(C.byref(handle), k, k, p(hm), p(hS), p(hL), p(hw), float(omega_f), float(tol),
                               C.byref(o), int(nthreads))
    check(rc, "pn_check_start")
    try:
        out = pn_integrate(m, S0, L0, omega0, omega_f, tol, o, out=out, stream=stream)
        idx = torch.from_numpy(sample).to(omega0.device)
        gy = np.ascontiguousarray(out["y"][:, idx].cpu().numpy())
        gs = np.ascontiguousarray(out["steps"][:, idx].cpu().numpy())
        gst = np.ascontiguousarray(out["status"][idx].cpu().numpy())
    except BaseException:
        load().pn_check_finish(handle, None, None, None, 0, 0.0, None, None)
        raise
    if dot_tol is None:
        dot_tol = 1e-8 if o.precision == _lib.PN_PREC_FP64 else 1e-3
    flags = np.zeros(k, dtype=np.int32)
    rep = _lib.PnCheckReport()
    rc = load().pn_check_finish(handle, p(gy), p(gs), p(gst), k, float(dot_tol), p(flags), C.byref(rep))
    check(rc, "pn_check_finish")
    report = {f: getattr(rep, f) for f, _ in _lib.PnCheckReport._fields_}
    report.update({"dot_tol": dot_tol, "sample": sample, "flags": flags, "ok": rep.flagged == 0})
    return out, report


def pn_integrate_noalloc(m, S0, L0, omega0, omega_f, tol, out: dict, opts: PnOpts | None = None,
                         stream=None) -> dict:
    """pn_integrate through the entry point that allocates no device memory
    (for graph capture and serving loops): `out` must be preallocated
    (alloc_outputs); the library uses a fixed scratch array of its own.
    Calls that overlap on one device race; calls on one stream are safe."""
    if out is None:
        raise ValueError("pn_integrate_noalloc needs preallocated outputs (alloc_outputs)")
    return _integrate("noalloc", m, S0, L0, omega0, omega_f, tol, opts, out, out.get("dots") is not None, stream)


def pn_integrate_phase(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, out=None,
                       dots: bool = True, stream=None) -> dict:
    """pn_integrate plus the orbital phase Phi = integral of omega dt at
    t_final: out["phase"] [n] float64.  Every other output is bit-identical
    to pn_integrate's."""
    return _integrate("phase", m, S0, L0, omega0, omega_f, tol, opts, out, dots, stream)


def _integrate(kind, m, S0, L0, omega0, omega_f, tol, opts, out, dots, stream) -> dict:
    n = int(omega0.shape[0])
    _soa(omega0, 1, n, "omega0")
    _soa(m, 2, n, "m"); _soa(S0, 6, n, "S0"); _soa(L0, 3, n, "L0")
    lds = {_ld(m, n), _ld(S0, n), _ld(L0, n)}
    if out is None:
        out = alloc_outputs(n, omega0.device, dots)
    for k, c in (("y", 10), ("steps", 3)):
        _soa(out[k], c, n, k, torch.int32 if k == "steps" else torch.float64)
        lds.add(_ld(out[k], n))
    _soa(out["t"], 1, n, "t"); _soa(out["status"], 1, n, "status", torch.int32)
    if out.get("dots") is not None:
        _soa(out["dots"], 3, n, "dots")
        lds.add(_ld(out["dots"], n))
    if kind == "phase":
        if out.get("phase") is None:
            out["phase"] = torch.empty((n,), dtype=torch.float64, device=omega0.device)
        _soa(out["phase"], 1, n, "phase")
    if n > 0 and len(lds) != 1:
        raise ValueError("all [components, n] arrays must share one leading dimension")
    ld = lds.pop() if n > 0 else 0
    o = opts if opts is not None else make_opts()
    p = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    args = (n, ld, p(m), p(S0), p(L0), p(omega0), float(omega_f), float(tol), C.byref(o), p(out["y"]),
            p(out["t"]), p(out["steps"]), p(out["status"]), p(out.get("dots")))
    if kind == "noalloc":
        rc = load().pn_integrate_noalloc(*args, _stream(stream))
        check(rc, "pn_integrate_noalloc")
    elif kind == "phase":
        rc = load().pn_integrate_phase(*args, p(out["phase"]), _stream(stream))
        check(rc, "pn_integrate_phase")
    else:
        rc = load().pn_integrate(*args, _stream(stream))
        check(rc, "pn_integrate")
    return out


def autotune(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, sample: int = 1 << 20,
             reps: int = 2, stream=None):
    """The fastest launch shape (refill threshold, block) of pn_integrate on
    the first `sample` inspirals; returns (opts, {(refill, block): ms}).
    Blocks until the timing runs are done."""
    n = int(omega0.shape[0])
    ns = n if sample <= 0 or sample > n else int(sample)
    _soa(omega0, 1, n, "omega0")
    _soa(m, 2, n, "m"); _soa(S0, 6, n, "S0"); _soa(L0, 3, n, "L0")
    lds = {_ld(m, n), _ld(S0, n), _ld(L0, n)}
    if n > 0 and len(lds) != 1:
        raise ValueError("all [components, n] arrays must share one leading dimension")
    ld = lds.pop() if n > 0 else 0
    out = {"y": torch.empty((10, ld), dtype=torch.float64, device=omega0.device),
           "t": torch.empty((ld,), dtype=torch.float64, device=omega0.device),
           "steps": torch.empty((3, ld), dtype=torch.int32, device=omega0.device),
           "status": torch.empty((ld,), dtype=torch.int32, device=omega0.device),
           "dots": torch.empty((3, ld), dtype=torch.float64, device=omega0.device)}
    best = PnOpts()
    times = (C.c_double * 8)()
    o = opts if opts is not None else make_opts()
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = load().pn_autotune(n, ld, p(m), p(S0), p(L0), p(omega0), float(omega_f), float(tol), C.byref(o), ns,
                            int(reps), p(out["y"]), p(out["t"]), p(out["steps"]), p(out["status"]), p(out["dots"]),
                            C.byref(best), times, _stream(stream))
    check(rc, "pn_autotune")
    table = {(r, b): times[i] for i, (r, b) in enumerate((r, b) for r in (2, 3, 4, 6) for b in (128, 256))}
    return best, table


def _check_inputs(m, S0, L0, omega0):
    n = int(omega0.shape[0])
    _soa(omega0, 1, n, "omega0")
    for t, c, name in ((m, 2, "m"), (S0, 6, "S0"), (L0, 3, "L0")):
        _soa(t, c, n, name)
        if n > 0 and _ld(t, n) != n:
            raise ValueError(f"{name} must be contiguous")
    return n


def pn_tape_stride(cap_steps: int, ckpt_every: int) -> int:
    return int(load().pn_tape_stride(int(cap_steps), int(ckpt_every)))


def pn_integrate_record(m, S0, L0, omega0, omega_f, tol, opts: PnOpts | None = None, *,
                        cap_steps: int = 4096, ckpt_every: int = 64, stream=None) -> dict:
    """pn_integrate that also writes the tape the adjoint replays (contiguous
    inputs).  Returns the outputs of pn_integrate plus 'tape' [n, stride]."""
    n = _check_inputs(m, S0, L0, omega0)
    out = alloc_outputs(n, omega0.device, True)
    stride = pn_tape_stride(cap_steps, ckpt_every)
    tape = torch.empty((n, stride), dtype=torch.float64, device=omega0.device)
    o = opts if opts is not None else make_opts()
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = load().pn_integrate_record(n, n, p(m), p(S0), p(L0), p(omega0), float(omega_f), float(tol),
                                    C.byref(o), p(out["y"]), p(out["t"]), p(out["steps"]),
                                    p(out["status"]), p(out["dots"]), p(tape), int(cap_steps),
                                    int(ckpt_every), _stream(stream))
    check(rc, "pn_integrate_record")
    out.update(tape=tape, cap_steps=int(cap_steps), ckpt_every=int(ckpt_every))
    return out


def pn_ckpt_bytes(n: int, cap_steps: int, ckpt_every: int) -> int:
    return int(load().pn_ckpt_bytes(int(n), int(cap_steps), int(ckpt_every)))


def pn_integrate_replay(m, S0, L0, omega0, omega_f, rec: dict, opts: PnOpts | None = None, stream=None) -> dict:
    """The recorded run's map with its step sizes frozen (rec: the dict of
    pn_integrate_record), evaluated at the initial state (m, S0, L0, omega0)
    (contiguous inputs).  Returns {'y': [10, n], 't': [n]}."""
    n = _check_inputs(m, S0, L0, omega0)
    if n != int(rec["tape"].shape[0]):
        raise ValueError("the tape must hold one row per inspiral")
    out = {"y": torch.empty((10, n), dtype=torch.float64, device=omega0.device),
           "t": torch.empty((n,), dtype=torch.float64, device=omega0.device)}
    o = opts if opts is not None else make_opts()
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = load().pn_integrate_replay(n, n, p(m), p(S0), p(L0), p(omega0), float(omega_f), C.byref(o),
                                    p(rec["tape"]), rec["cap_steps"], rec["ckpt_every"], p(rec["status"]),
                                    p(out["y"]), p(out["t"]), _stream(stream))
    check(rc, "pn_integrate_replay")
    return out


def pn_integrate_adjoint(m, omega_f, rec: dict, gy, gt=None, opts: PnOpts | None = None,
                         order=None, stream=None) -> dict:
    """Gradients of sum(gy * y_final) + sum(gt * t_final) with respect to
    m [2, n], S0 [6, n], L0 [3, n], omega0 [n], for the recorded run `rec`
    (the dict returned by pn_integrate_record)."""
    n = int(rec["status"].shape[0])
    _soa(m, 2, n, "m"); _soa(gy, 10, n, "gy")
    if gt is not None:
        _soa(gt, 1, n, "gt")
    if n > 0 and (_ld(m, n) != n or _ld(gy, n) != n):
        raise ValueError("m and gy must be contiguous (leading dimension n)")
    if order is not None:
        _soa(order, 1, n, "order", torch.int32)
    K = rec["ckpt_every"]
    dev = m.device
    ws_bytes = int(load().pn_adjoint_workspace_bytes(n, K))
    ws = torch.empty(max(ws_bytes // 8, 1), dtype=torch.float64, device=dev)
    g = {"m": torch.empty((2, n), dtype=torch.float64, device=dev),
         "S0": torch.empty((6, n), dtype=torch.float64, device=dev),
         "L0": torch.empty((3, n), dtype=torch.float64, device=dev),
         "omega0": torch.empty((n,), dtype=torch.float64, device=dev)}
    o = opts if opts is not None else make_opts()
    p = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    rc = load().pn_integrate_adjoint(n, n, p(m), float(omega_f), C.byref(o), p(rec["tape"]),
                                     rec["cap_steps"], K, p(rec["status"]), p(gy), p(gt), p(g["m"]),
                                     p(g["S0"]), p(g["L0"]), p(g["omega0"]), p(ws), ws_bytes, p(order),
                                     _stream(stream))
    check(rc, "pn_integrate_adjoint")
    return g


class PNIntegrate(torch.autograd.Function):
    """y_final, t_final = PNIntegrate.apply(m, S0, L0, omega0, omega_f, tol, ckpt_every, cap_steps)

    Forward: the recorded FP64 integration.  Backward: the discrete adjoint
    with the accepted step sizes held fixed.  Inputs contiguous on the GPU.
    A run that needs more than cap_steps accepted steps is repeated with a
    doubled cap."""

    @staticmethod
    def forward(ctx, m, S0, L0, omega0, omega_f, tol, ckpt_every=64, cap_steps=2048):
        m, S0, L0, omega0 = (t.detach().contiguous() for t in (m, S0, L0, omega0))
        cap = int(cap_steps)
        while True:
            rec = pn_integrate_record(m, S0, L0, omega0, omega_f, tol, cap_steps=cap,
                                      ckpt_every=int(ckpt_every))
            if not bool((rec["status"] == _lib.PN_ST_TAPE_FULL).any()):
                break
            cap *= 2
        ctx.rec = rec
        ctx.omega_f = float(omega_f)
        ctx.save_for_backward(m)
        ctx.mark_non_differentiable(rec["status"], rec["steps"])
        return rec["y"], rec["t"], rec["status"], rec["steps"]

    @staticmethod
    def backward(ctx, gy, gt, _gs, _gst):
        (m,) = ctx.saved_tensors
        rec = ctx.rec
        gy = torch.zeros_like(rec["y"]) if gy is None else gy.contiguous()
        gt = None if gt is None else gt.contiguous()
        order = torch.argsort(rec["steps"][0], descending=True).to(torch.int32)
        g = pn_integrate_adjoint(m, ctx.omega_f, rec, gy, gt, order=order)
        return g["m"], g["S0"], g["L0"], g["omega0"], None, None, None, None


def pn_shutdown() -> None:
    """Free the library's context on the current device (call slots); only
    when none of its work is pending (synchronize first)."""
    check(load().pn_shutdown(), "pn_shutdown")


def pn_fma_lanes(active_lanes: int, iters: int = 4000, stream=None) -> dict:
    """One launch of FP64 FMA chains on the first active_lanes lanes of every
    wave (one wave per SIMD): its lane FLOPs and duration."""
    flop, ms = C.c_double(), C.c_double()
    rc = load().pn_fma_lanes(int(active_lanes), int(iters), C.byref(flop), C.byref(ms), _stream(stream))
    check(rc, "pn_fma_lanes")
    return {"active_lanes": int(active_lanes), "lane_flop": flop.value, "ms": ms.value}


def pn_fma_rate(waves_per_simd: int = 8, iters: int = 4000, stream=None) -> dict:
    """Sustained vector FMA rate of the current device in TFLOP/s: FP32
    without packed instructions, and FP64 (blocks until measured)."""
    f32, f64 = C.c_double(0.0), C.c_double(0.0)
    rc = load().pn_fma_rate(int(waves_per_simd), int(iters), C.byref(f32), C.byref(f64), _stream(stream))
    check(rc, "pn_fma_rate")
    return {"fp32_nonpacked": f32.value, "fp64": f64.value, "unit": "TFLOP/s", "waves_per_simd": int(waves_per_simd)}


def pn_rhs(m, y, opts: PnOpts | None = None, stream=None) -> torch.Tensor:
    """Eqs. (1)-(4) pointwise: m [2, n], y [10, n] -> dy/dt [10, n]."""
    n = int(y.shape[1])
    _soa(m, 2, n, "m"); _soa(y, 10, n, "y")
    if _ld(m, n) != _ld(y, n):
        raise ValueError("m and y must share one leading dimension")
    out = torch.empty((10, n), dtype=torch.float64, device=y.device)
    if _ld(out, n) != _ld(y, n):
        raise ValueError("y must be contiguous")
    o = opts if opts is not None else make_opts()
    rc = load().pn_rhs(n, _ld(y, n), C.c_void_p(m.data_ptr()), C.c_void_p(y.data_ptr()),
                       C.c_void_p(out.data_ptr()), C.byref(o), _stream(stream))
    check(rc, "pn_rhs")
    return out


def pn_observables(y, stream=None) -> torch.Tensor:
    """(S1_hat.S2_hat, S1_hat.L_hat, S2_hat.L_hat) of states y [10, n] -> [3, n]."""
    n = int(y.shape[1])
    _soa(y, 10, n, "y")
    out = torch.empty((3, n), dtype=torch.float64, device=y.device)
    if _ld(out, n) != _ld(y, n):
        raise ValueError("y must be contiguous")
    rc = load().pn_observables(n, _ld(y, n), C.c_void_p(y.data_ptr()), C.c_void_p(out.data_ptr()),
                               _stream(stream))
    check(rc, "pn_observables")
    return out


# ---------------------------------------------------------------------------
# the statistics of Sec. V
# ---------------------------------------------------------------------------

def _comp(x, name):
    """A [ncomp, n] float64 device array with unit stride along n."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    _on_current_device(x, name)
    if x.dim() == 1:
        x = x.unsqueeze(0)
    if x.dtype != torch.float64 or x.dim() != 2 or (x.shape[1] > 1 and x.stride(1) != 1):
        raise ValueError(f"{name} must be a float64 [ncomp, n] array with unit stride along n")
    return x


def pn_histogram(x, nbins=20, lo=-1.0, hi=1.0, stream=None) -> torch.Tensor:
    """Counts [ncomp, nbins] (int64) of x [ncomp, n] in equal bins on [lo, hi]."""
    x = _comp(x, "x")
    nc, n = int(x.shape[0]), int(x.shape[1])
    out = torch.empty((nc, nbins), dtype=torch.int64, device=x.device)
    rc = load().pn_histogram(n, _ld(x, n) if n else 0, C.c_void_p(x.data_ptr()), nc, int(nbins), float(lo),
                             float(hi), C.c_void_p(out.data_ptr()), _stream(stream))
    check(rc, "pn_histogram")
    return out


def pn_histogram2d(x, y, nbins=79, lo=-1.0, hi=1.0, stream=None) -> torch.Tensor:
    """Bivariate counts [ncomp, nbins (x), nbins (y)] (int64)."""
    x, y = _comp(x, "x"), _comp(y, "y")
    nc, n = int(x.shape[0]), int(x.shape[1])
    if tuple(y.shape) != tuple(x.shape) or (n and _ld(x, n) != _ld(y, n)):
        raise ValueError("x and y must have one shape and leading dimension")
    out = torch.empty((nc, nbins, nbins), dtype=torch.int64, device=x.device)
    rc = load().pn_histogram2d(n, _ld(x, n) if n else 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nc,
                               int(nbins), float(lo), float(hi), C.c_void_p(out.data_ptr()), _stream(stream))
    check(rc, "pn_histogram2d")
    return out


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=device)


def pn_pearson(x, y, stream=None) -> torch.Tensor:
    """[ncomp, 5]: mean x, mean y, std x, std y (1/(n-1)), Pearson r."""
    x, y = _comp(x, "x"), _comp(y, "y")
    nc, n = int(x.shape[0]), int(x.shape[1])
    if tuple(y.shape) != tuple(x.shape) or (n and _ld(x, n) != _ld(y, n)):
        raise ValueError("x and y must have one shape and leading dimension")
    out = torch.empty((nc, 5), dtype=torch.float64, device=x.device)
    wb = int(load().pn_stats_workspace_bytes(n, nc, 0))
    ws = _workspace(wb, x.device)
    rc = load().pn_pearson(n, _ld(x, n) if n else 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nc,
                           C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), wb, _stream(stream))
    check(rc, "pn_pearson")
    return out


def pn_kde(x, sigma, ngrid=201, lo=-1.0, hi=1.0, stream=None) -> torch.Tensor:
    """Gaussian KDE [ncomp, ngrid] on lo + k (hi - lo)/(ngrid - 1), bandwidth
    1.06 sigma n^(-1/5); sigma: device [ncomp] (e.g. pn_pearson(...)[:, 2])."""
    x = _comp(x, "x")
    nc, n = int(x.shape[0]), int(x.shape[1])
    if not isinstance(sigma, torch.Tensor) or sigma.dtype != torch.float64 or sigma.numel() != nc \
            or sigma.device != x.device:
        raise ValueError("sigma must be a float64 device array of ncomp values")
    out = torch.empty((nc, ngrid), dtype=torch.float64, device=x.device)
    wb = int(load().pn_stats_workspace_bytes(n, nc, ngrid))
    ws = _workspace(wb, x.device)
    rc = load().pn_kde(n, _ld(x, n) if n else 0, C.c_void_p(x.data_ptr()), nc, C.c_void_p(sigma.data_ptr()),
                       int(sigma.stride(0)) if sigma.dim() == 1 else 1, int(ngrid), float(lo), float(hi),
                       C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), wb, _stream(stream))
    check(rc, "pn_kde")
    return out


def pn_ks_uniform(x, lo=-1.0, hi=1.0, stream=None) -> torch.Tensor:
    """[ncomp, 2]: the K-S statistic D against U[lo, hi] and its asymptotic p-value."""
    x = _comp(x, "x")
    nc, n = int(x.shape[0]), int(x.shape[1])
    out = torch.empty((nc, 2), dtype=torch.float64, device=x.device)
    wb = int(load().pn_ks_workspace_bytes(n))
    ws = _workspace(wb, x.device)
    rc = load().pn_ks_uniform(n, _ld(x, n) if n else 0, C.c_void_p(x.data_ptr()), nc, float(lo), float(hi),
                              C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), wb, _stream(stream))
    check(rc, "pn_ks_uniform")
    return out


def statistics(dots_initial, dots_final, nbins=20, nbins2d=79, ngrid=201, stream=None) -> dict:
    """The statistics of Sec. V for the three unit-vector dot products:
    histograms of the final values, the bivariate histograms and Pearson r of
    initial against final, the KDE and the K-S test of the final values."""
    p = pn_pearson(dots_initial, dots_final, stream=stream)
    return {"hist": pn_histogram(dots_final, nbins, stream=stream),
            "hist2d": pn_histogram2d(dots_initial, dots_final, nbins2d, stream=stream),
            "pearson": p,
            "kde": pn_kde(dots_final, p[:, 3].contiguous(), ngrid, stream=stream),
            "ks": pn_ks_uniform(dots_final, stream=stream)}


def initial_dots(d: dict, stream=None) -> torch.Tensor:
    """The dot products of the initial states of device inputs d (to_device)."""
    y0 = torch.cat([d["omega0"][None], d["S"], d["L"]], 0).contiguous()
    return pn_observables(y0, stream=stream)


def pearson_study(kind: str, values, n: int = 16384, base="paper_equal_mass", m1: float | None = None,
                  chi: float | None = None, stream=None) -> dict:
    """The parameter studies of Sec. V B-D: for each value, a population of n
    inspirals of the base workload (a name in population.WORKLOADS or a
    Workload) with m1 = value (chi_1 = chi_2 = 1), chi_1 = chi_2 = value
    (m1 = m2), omega0 = value or omega_f = value, integrated on the GPU, and
    the Pearson r of initial against final S1.S2, S1.L, S2.L.  m1 and chi, if
    given, are held at those values first (for instance m1 = 0.4, chi = 0.05,
    the case of Sec. V D whose correlations depend on omega0 and omega_f).
    Returns {"values", "r" [k, 3], "ok" [k]}."""
    import dataclasses

    import numpy as np

    from . import population
    w0 = base if isinstance(base, population.Workload) else population.WORKLOADS[base]
    if m1 is not None:
        w0 = dataclasses.replace(w0, q=("fixed", float(m1) / (1.0 - float(m1))))
    if chi is not None:
        w0 = dataclasses.replace(w0, chi=("fixed", float(chi), float(chi)))
    rs, oks = [], []
    for v in values:
        if kind == "m1":
            w = dataclasses.replace(w0, q=("fixed", float(v) / (1.0 - float(v))), chi=("fixed", 1.0, 1.0))
        elif kind == "chi":
            w = dataclasses.replace(w0, q=("fixed", 1.0), chi=("fixed", float(v), float(v)))
        elif kind == "omega0":
            w = dataclasses.replace(w0, omega0=("fixed", float(v)))
        elif kind == "omega_f":
            w = dataclasses.replace(w0, omega_f=float(v))
        else:
            raise ValueError("kind is 'm1', 'chi', 'omega0' or 'omega_f'")
        pop = population.generate(w, n)
        d = to_device(pop)
        out = pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], stream=stream)
        r = pn_pearson(initial_dots(d, stream=stream), out["dots"], stream=stream)[:, 4]
        rs.append(r.cpu().numpy())
        oks.append(bool((out["status"] == 0).all()))
    return {"values": list(map(float, values)), "r": np.array(rs), "ok": oks}


def gen_spec(q=(1.0, 1.0), chi1=(1.0, 1.0), chi2=(1.0, 1.0), omega0=(0.01, 0.01), seed=0) -> "_lib.PnGenSpec":
    """The distribution pn_generate draws from: (lo, hi) per parameter, fixed
    when lo == hi."""
    return _lib.PnGenSpec(float(q[0]), float(q[1]), float(chi1[0]), float(chi1[1]), float(chi2[0]),
                          float(chi2[1]), float(omega0[0]), float(omega0[1]), int(seed))


def pn_generate(n: int, spec, first: int = 0, device="cuda", out=None, stream=None) -> dict:
    """Inspirals first .. first + n - 1 of the Philox population `spec`
    (gen_spec) drawn on the GPU: dict(m [2, n], S [6, n], L [3, n], omega0 [n])."""
    if out is None:
        out = {"m": torch.empty((2, n), dtype=torch.float64, device=device),
               "S": torch.empty((6, n), dtype=torch.float64, device=device),
               "L": torch.empty((3, n), dtype=torch.float64, device=device),
               "omega0": torch.empty((n,), dtype=torch.float64, device=device)}
    for k, c in (("m", 2), ("S", 6), ("L", 3)):
        _soa(out[k], c, n, k)
    _soa(out["omega0"], 1, n, "omega0")
    lds = {_ld(out[k], n) for k in ("m", "S", "L")} if n else {0}
    if len(lds) != 1:
        raise ValueError("the output arrays must share one leading dimension")
    rc = load().pn_generate(n, lds.pop(), int(first), C.byref(spec), C.c_void_p(out["m"].data_ptr()),
                            C.c_void_p(out["S"].data_ptr()), C.c_void_p(out["L"].data_ptr()),
                            C.c_void_p(out["omega0"].data_ptr()), _stream(stream))
    check(rc, "pn_generate")
    return out


def ks_run(total: int, spec, omega_f: float, tol: float, chunk: int = 1 << 22, nbins: int = 100,
           stream=None) -> dict:
    """The K-S test of Sec. V at scale, streamed on the GPU: chunks of
    generate -> integrate, keeping only the final S1_hat.S2_hat of every
    inspiral (8 B each), then the K-S statistic against U[-1, 1] and a
    histogram over the whole sample.  No host traffic but the results."""
    dev = "cuda"
    chunk = min(chunk, total)
    keep = torch.empty((1, total), dtype=torch.float64, device=dev)
    pop = pn_generate(chunk, spec, 0, dev, stream=stream)
    out = alloc_outputs(chunk, dev)
    bad = torch.zeros((), dtype=torch.int64, device=dev)
    for first in range(0, total, chunk):
        n = min(chunk, total - first)
        if n < chunk:
            pop = {k: v[..., :n] for k, v in pop.items()}
            out = {k: (v[..., :n] if v is not None else None) for k, v in out.items()}
        pn_generate(n, spec, first, dev, out=pop, stream=stream)
        pn_integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], omega_f, tol, out=out, stream=stream)
        keep[0, first:first + n].copy_(out["dots"][0])
        bad += (out["status"] != 0).sum()
    return {"n": total, "ks": pn_ks_uniform(keep, stream=stream)[0], "hist": pn_histogram(keep, nbins, stream=stream)[0],
            "not_ok": bad, "final_s1s2": keep[0]}


def to_device(pop: dict, device="cuda") -> dict:
    """The input arrays of a population (numpy, from population.generate) on the GPU."""
    return {k: torch.from_numpy(pop[k]).to(device) for k in ("m", "S", "L", "omega0")}
