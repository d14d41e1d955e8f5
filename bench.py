"""Throughput benchmark of the gfx950 post-Newtonian inspiral integrator.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload q1to4_1M]

One step = one pn_integrate call over the whole workload: every inspiral
integrated from omega0 to omega_f with adaptive Dormand-Prince at the
workload's tolerance, outputs written to HBM (final state, time, step counts,
status, the three unit-vector dot products).  Inputs are already resident on
the GPU when the timed region starts.  Prints one JSON line.

The default workload is 1,048,576 inspirals, q = m1/m2 ~ U[1,4], M = 1,
chi_i ~ U[0,1], isotropic spin directions, L_hat = z, M omega 0.005 -> 0.05,
FP64, tol 1e-8 (synthetic, seeded).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "inspirals/s to ω_f at 1e-8 tol; RHS evals/s as % VALU peak; adjoint/fwd cost"

# Algorithmic work per unit: the arithmetic of Eqs. (1)-(4) and of the
# Dormand-Prince tableau with each operation written once, a fused
# multiply-add counted as 2 FLOP and a division as 1; the cube root, the log
# and err^(-1/5) are special functions and not counted.  One right-hand-side
# evaluation (F_RHS) and the stage sums, error estimate, error norm and step
# control of one attempted step (F_STEP_COMB).  RHS_FLOP and COMB_FLOP list
# the terms; tests check that they add up.
RHS_FLOP = {
    "v = M w, x^2": 2,
    "L.S1, L.S2, S1.S2 (2 FMA + 1 MUL each)": 15,
    "3.5PN bracket: spin-orbit (2 FMA), spin-spin (2 MUL + FMA), c4', c6' (FMA each)": 12,
    "Horner chain in x (6 FMA)": 12,
    "d omega/dt = K w^2 x^2 v B (5 MUL)": 5,
    "p = w/2, s_v = w/M, -3 s_v": 3,
    "alpha_1, alpha_2 (MUL + FMA + MUL each), beta": 9,
    "Omega_1, Omega_2 (3 MUL + 3 FMA each)": 18,
    "Omega_1 x S1, Omega_2 x S2 (3 MUL + 3 FMA each)": 18,
    "dL/dt = -lambda x (dS1 + dS2) (MUL, 3 ADD, 3 MUL)": 7,
}
COMB_FLOP = {
    "stage points Y_2..Y_7: 20 nonzero a_sj x 10 components (FMA)": 400,
    "h a_sj products": 20,
    "error estimate sum_j (b_j - bhat_j) k_j: 10 x (MUL + 5 FMA)": 110,
    "error norm: 10 x (scale FMA, division, square-add FMA), x 0.1 h^2": 53,
    "step factor 0.9 p, h fac, t + h": 3,
}
F_RHS = sum(RHS_FLOP.values())            # 101
F_STEP_COMB = sum(COMB_FLOP.values())     # 586
# The oracle's own counts (its counting scalar: every add, sub, mul and div of
# its deliberately plain association, one FLOP each) and the per-attempted-step
# estimate of the hot-path plan, reported beside the fraction for comparison.
ORACLE_F_RHS = 134
ORACLE_F_STEP_COMB = 704
PLAN_F_STEP = 1300
FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X: 256 CU x 2.4 GHz x 128 FLOP/clk
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X datasheet (counts packed FP32; the library is
                                    # compiled without packed FP32 instructions, so half of
                                    # it is the reachable ceiling)
HBM_PEAK_GBS = 8000.0


def algorithmic_flops(steps: np.ndarray, f_rhs: int = F_RHS, f_comb: int = F_STEP_COMB) -> float:
    """FLOPs of the method for step counts [3, n] (accepted, rejected, RHS evals):
    every attempted step costs 6 RHS evaluations + one combination; the first
    RHS evaluation of each inspiral is extra."""
    nrhs = steps[2].astype(np.int64)
    attempted = (nrhs - 1) // 6
    return float((nrhs * f_rhs).sum() + (attempted * f_comb).sum())


def attempted_steps(steps: np.ndarray) -> int:
    return int(((steps[2].astype(np.int64) - 1) // 6).sum())


def cpu_baseline(pop: dict, budget_s: float = 12.0, gpu: dict | None = None, dot_tol: float = 1e-8) -> dict:
    """The oracle, as it stands, on a bounded prefix of the same workload,
    on every host core this process may use.  With the GPU's outputs for the
    population (`gpu`: numpy dots [3, n], steps [3, n], status [n]) the
    sample is also compared with them, as the paper checked its GPU runs
    against the CPU on a subset (Sec. III): statuses, accepted and rejected
    step counts, and the final dot products to dot_tol."""
    import oracle
    from paper_0908_3889_amd import population as P

    cores = len(os.sched_getaffinity(0))
    probe = min(pop["n"], 2048)
    sub = P.subset(pop, np.arange(probe))
    t0 = time.perf_counter()
    oracle.integrate(sub["m"], sub["S"], sub["L"], sub["omega0"], pop["omega_f"], pop["tol"],
                     nthreads=cores)
    dt = time.perf_counter() - t0
    n_s = int(min(pop["n"], max(probe, probe * budget_s / max(dt, 1e-6))))
    sub = P.subset(pop, np.arange(n_s))
    t0 = time.perf_counter()
    r = oracle.integrate(sub["m"], sub["S"], sub["L"], sub["omega0"], pop["omega_f"], pop["tol"],
                         nthreads=cores)
    dt = time.perf_counter() - t0
    res = {"value": n_s / dt, "unit": "inspirals/s", "cores": cores, "kind": "oracle",
           "sample": f"first {n_s} of {pop['n']} inspirals of {pop['workload']}, {dt:.1f} s",
           "rhs_evals_per_s": float(r["steps"][2].sum()) / dt}
    # one host core on a small part of the same sample (about a tenth of the budget)
    n1 = int(max(1, min(n_s, n_s / dt * budget_s / 10 / max(cores, 1))))
    one = P.subset(pop, np.arange(n1))
    t0 = time.perf_counter()
    oracle.integrate(one["m"], one["S"], one["L"], one["omega0"], pop["omega_f"], pop["tol"], nthreads=1)
    res["per_core"] = {"value": n1 / (time.perf_counter() - t0), "sample": f"first {n1} inspirals, one thread"}
    if gpu is not None:
        res["crosscheck"] = crosscheck(r, {k: v[..., :n_s] for k, v in gpu.items()}, dot_tol)
    return res


def crosscheck(ref: dict, gpu: dict, dot_tol: float) -> dict:
    """GPU outputs against the oracle's on the same inspirals."""
    import oracle
    dots = oracle.observables(ref["y"])
    both = (ref["status"] == 0) & (gpu["status"] == 0)
    dd = np.abs(gpu["dots"][:, both] - dots[:, both])
    max_dd = float(dd.max()) if dd.size else 0.0
    status_diff = int((ref["status"] != gpu["status"]).sum())
    steps_diff = int(((ref["steps"][0] != gpu["steps"][0]) | (ref["steps"][1] != gpu["steps"][1])).sum())
    return {"n": int(ref["status"].size), "status_mismatches": status_diff, "step_count_mismatches": steps_diff,
            "max_dot_diff": max_dd, "dot_tol": dot_tol, "ok": bool(status_diff == 0 and max_dd < dot_tol)}


PROFILES = os.path.join(ROOT, "profiles")
COPY_CAL_BYTES = 512 << 20


def _profile_field(path: str, key: str):
    """A numeric field of a committed counter summary, or None when the file
    is missing or the device sources have changed since it was taken."""
    from paper_0908_3889_amd import build
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_digest") != build.source_digest():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def measured_counter_flop(kernel: str, workload: str):
    """FP64 lane FLOPs executed per launch of `kernel` on `workload`, from the
    committed summary profiles/flops_<kernel>_<workload>.txt (rocprofv3's
    SQ_INSTS_VALU_FLOPS_FP64 times the active lanes per VALU instruction,
    calibrated on launches with a known number of active lanes)."""
    return _profile_field(os.path.join(PROFILES, f"flops_{kernel}_{workload}.txt"), "counter_flop_per_launch")


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload`, from the committed
    counter summary profiles/hbm_<kernel>_<workload>.txt (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a plain copy of known
    size).  None when there is no such summary or the device sources have
    changed since the counters were taken."""
    return _profile_field(os.path.join(PROFILES, f"hbm_{kernel}_{workload}.txt"), "hbm_bytes_per_launch")


def kernel_resources(kernel: str, block: int):
    """VGPRs, AGPRs, spills, scratch, LDS and occupancy of the timed kernel
    instantiation, from the compiler's resource report of the build."""
    from paper_0908_3889_amd import build
    want = {"integrate_persistent_f64": f"integrate_persistent_f64ILi{block}ELb0E",
            "integrate_persistent_f32s": f"integrate_persistent_f32sILi{block}E",
            "integrate_static_f64": f"integrate_static_f64ILi{block}ELb0E",
            "integrate_static_f32s": f"integrate_static_f32sILi{block}E",
            "integrate_persistent_f32x": f"integrate_persistent_f32xILi{block}E",
            "integrate_static_f32x": f"integrate_static_f32xILi{block}E"}.get(kernel)
    if kernel.endswith("_phase"):
        want = f"{kernel}ILi{block}E"
    for name, fields in build.resource_usage().items():
        if want and want in name:
            keep = ("VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]", "VGPRs Spill",
                    "SGPRs Spill", "LDS Size [bytes/block]")
            return {k: int(fields[k]) for k in keep if k in fields and fields[k].lstrip("-").isdigit()}
    return None


def calibrate_copy() -> int:
    """Three device-to-device copies of COPY_CAL_BYTES each (the reference
    kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    a = torch.ones(COPY_CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_CAL_BYTES, "copies": 3}), flush=True)
    return 0


def calibrate_lanes() -> int:
    """FP64 FMA chains on 64, 32, 16, 4 and 1 active lanes per wave, one launch
    each in that order (the reference launches for reading FLOP and
    thread-cycle counters on partly active waves)."""
    from paper_0908_3889_amd import api
    runs = [api.pn_fma_lanes(k, 2000) for k in (64, 32, 16, 4, 1)]
    print(json.dumps({"calibrate_lanes": runs}), flush=True)
    return 0


def _time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def _time_calls(fn, reps: int, stream) -> float:
    """Mean time (ms) per call of `reps` back-to-back calls of fn, between two
    HIP events on the launch stream (after one untimed call)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _frac(steps: np.ndarray, ms: float, peak: float) -> float:
    return algorithmic_flops(steps) / (ms * 1e-3) / 1e12 / peak


def _stats(x: np.ndarray) -> dict:
    x = np.asarray(x, dtype=np.float64)
    return {"max": float(x.max()), "p99": float(np.percentile(x, 99))}


def leg_adjoint(api, population, stream, ks=(16, 64, 256), reps: int = 5, n: int | None = None) -> dict:
    """The differentiation workload (65,536 inspirals, tol 1e-8): the plain
    forward, the forward that records the tape (r_ckpt) and the discrete
    adjoint of loss = sum S1.S2 + sum L_hat_z (r_bwd), per checkpoint
    spacing K, each against the plain forward."""
    import torch
    w = population.WORKLOADS["adjoint_64k"]
    pop = population.generate(w, n)
    d = api.to_device(pop)
    out = api.alloc_outputs(pop["n"])
    fwd = lambda: api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], out=out,
                                   stream=stream)
    t_fwd = _time_calls(fwd, reps, stream)
    res = {"workload": w.name, "n": pop["n"], "tol": w.tol, "loss": "sum S1.S2 + sum L_hat_z (final)",
           "fwd_ms": t_fwd, "per_K": {},
           "timing": f"HIP events around {reps} back-to-back calls on the launch stream"}
    for K in ks:
        box = {}

        def rec():
            box["rec"] = api.pn_integrate_record(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"],
                                                 pop["tol"], cap_steps=1024, ckpt_every=K, stream=stream)
        t_rec = _time_calls(rec, reps, stream)
        r = box["rec"]
        y = r["y"]
        gy = torch.zeros_like(y)
        gy[1:4] = y[4:7]
        gy[4:7] = y[1:4]
        gy[9] = 1.0
        order = torch.argsort(r["steps"][0], descending=True).to(torch.int32)

        def adj():
            box["g"] = api.pn_integrate_adjoint(d["m"], pop["omega_f"], r, gy, order=order, stream=stream)
        t_adj = _time_calls(adj, reps, stream)
        res["per_K"][str(K)] = {"record_ms": t_rec, "adjoint_ms": t_adj, "r_ckpt": t_rec / t_fwd,
                                "r_bwd": t_adj / t_fwd, "r_total": (t_rec + t_adj) / t_fwd,
                                "ok": int((r["status"] == 0).sum().item()),
                                "grad_finite": bool(torch.isfinite(box["g"]["S0"]).all().item())}
    res["r_bwd_max"] = max(v["r_bwd"] for v in res["per_K"].values())
    return res


def _ordered_run(api, pop, d, opts, out, stream, order: bool = True):
    """One integration of the population, the longest-first hand-out order
    (pn_cost_order) computed first when `order`."""
    import torch
    if not order:
        api.set_order(opts, None)
        api.set_packed(opts, None)
        return lambda: api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                                        out=out, stream=stream)
    buf = torch.empty((pop["n"],), dtype=torch.int32, device="cuda")
    ws = api.cost_order_workspace(pop["n"])
    packed = api.packed_inputs(pop["n"])
    api.set_order(opts, buf)
    api.set_packed(opts, packed)

    def run():
        api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], out=buf, workspace=ws,
                          packed=packed, stream=stream)
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts, out=out,
                         stream=stream)
    return run


def leg_fp32split(api, pop, d, ref64: dict, stream, reps: int = 5, precision: str = "fp32split") -> dict:
    """An FP32 mode (FP32-split: FP64 state; "fp32": FP32 state with
    compensated omega and phase) on the same population as the FP64 run:
    time, fraction of the FP32 vector peak, and the error of every output
    against the FP64 path (which the CPU-baseline leg checks against the
    oracle)."""
    import torch
    opts = api.make_opts(precision=precision)
    out = api.alloc_outputs(pop["n"])
    run = _ordered_run(api, pop, d, opts, out, stream)
    ms = _time_calls(run, reps, stream)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    ok = (g["status"] == 0) & (ref64["status"] == 0)
    S0 = pop["S"]
    n1 = np.linalg.norm(S0[:3], axis=0)
    n2 = np.linalg.norm(S0[3:], axis=0)
    n1[n1 == 0] = 1.0
    n2[n2 == 0] = 1.0
    y, y64 = g["y"][:, ok], ref64["y"][:, ok]
    err = {
        "S1h.S2h": _stats(np.abs(g["dots"][0] - ref64["dots"][0])[ok]),
        "S1h.Lh": _stats(np.abs(g["dots"][1] - ref64["dots"][1])[ok]),
        "S2h.Lh": _stats(np.abs(g["dots"][2] - ref64["dots"][2])[ok]),
        "S1 (|dS1|/|S1(0)|)": _stats(np.linalg.norm(y[1:4] - y64[1:4], axis=0) / n1[ok]),
        "S2 (|dS2|/|S2(0)|)": _stats(np.linalg.norm(y[4:7] - y64[4:7], axis=0) / n2[ok]),
        "L_hat (|dL|)": _stats(np.linalg.norm(y[7:10] - y64[7:10], axis=0)),
        "t (relative)": _stats(np.abs(g["t"][ok] / ref64["t"][ok] - 1)),
    }
    # the orbital phase, integrated alongside in both precisions (untimed)
    api.set_order(opts, None)
    api.set_packed(opts, None)
    p32 = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                                 stream=stream)
    p64 = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                 stream=stream)
    torch.cuda.synchronize()
    ph32, ph64 = p32["phase"].cpu().numpy()[ok], p64["phase"].cpu().numpy()[ok]
    err["phase (relative)"] = _stats(np.abs(ph32 / ph64 - 1))
    return {"ms": ms, "frac": _frac(g["steps"], ms, FP32_VECTOR_PEAK_TFLOPS),
            "frac_of_nonpacked_fp32": _frac(g["steps"], ms, FP32_VECTOR_PEAK_TFLOPS / 2),
            "status_ok": int((g["status"] == 0).sum()), "n": pop["n"],
            "steps_equal_to_fp64": float((g["steps"][:2] == ref64["steps"][:2]).all(axis=0).mean()),
            "error_vs_fp64": err,
            "reference": "the FP64 path on the whole population (its own distance from the oracle is "
                         "cpu_baseline.crosscheck)"}


def leg_check(api, pop, d, stream, fractions=(0.001, 0.01)) -> dict:
    """The CPU check of Sec. III as the library runs it (integrate_checked):
    a random fraction of the population integrated on the host threads while
    the GPU integrates all of it, then compared at the 1e-8 parity bar.  Wall
    time of the checked call against the GPU integration alone."""
    import torch
    cores = len(os.sched_getaffinity(0))
    res = {"workload": pop["workload"], "n": pop["n"], "host_threads": cores, "runs": []}
    for f in fractions:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = api.integrate_checked(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                       fraction=f, seed=11, host_inputs=pop, nthreads=cores, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res["runs"].append({"fraction": f, "checked": rep["checked"], "wall_ms": wall * 1e3,
                            "host_ms": rep["host_seconds"] * 1e3, "flagged": rep["flagged"],
                            "status_mismatches": rep["status_mismatches"],
                            "step_mismatches": rep["step_mismatches"], "max_dot_diff": rep["max_dot_diff"],
                            "ok": rep["ok"]})
    return res


def leg_batching(api, population, stream, reps: int = 3, n: int | None = None) -> dict:
    """The batching workload (4,194,304 inspirals, omega0 log-uniform in
    [0.002, 0.01], q in [1, 10]): the persistent refill kernel against one
    lane per inspiral without refill (in index order), and the persistent
    kernel with the inspirals handed out longest first (pn_cost_order,
    timed with it)."""
    w = population.WORKLOADS["batching_4M"]
    pop = population.generate(w, n)
    d = api.to_device(pop)
    out = api.alloc_outputs(pop["n"])
    res = {"workload": w.name, "n": pop["n"]}
    for name, sched, order in (("persistent_cost_order", "persistent", True),
                               ("persistent", "persistent", False), ("static", "static", False)):
        opts = api.make_opts(schedule=sched)
        run = _ordered_run(api, pop, d, opts, out, stream, order)
        ms = _time_calls(run, reps, stream)
        steps = out["steps"].cpu().numpy()
        res[name] = {"ms": ms, "inspirals_per_s": pop["n"] / (ms * 1e-3),
                     "frac": _frac(steps, ms, FP64_VECTOR_PEAK_TFLOPS),
                     "status_ok": int((out["status"] == 0).sum().item())}
    acc = steps[0].astype(np.int64)
    res["accepted_steps_min_median_max"] = [int(acc.min()), int(np.median(acc)), int(acc.max())]
    res["static_over_persistent"] = res["static"]["ms"] / res["persistent"]["ms"]
    res["static_over_persistent_cost_order"] = res["static"]["ms"] / res["persistent_cost_order"]["ms"]
    return res


def bench_adjoint(args, api, pop, d, w, step, stream) -> int:
    """Cost of the recorded forward and of the discrete adjoint relative to
    the plain forward, per checkpoint spacing K (one JSON line)."""
    import torch
    t_fwd = _time(step, args.steps, args.warmup, stream)
    out = {"metric": "adjoint/fwd cost", "workload": w.name, "n": pop["n"], "tol": w.tol,
           "loss": "sum S1.S2 + sum L_hat_z (final)", "fwd_ms": t_fwd, "per_K": {}}
    for K in [int(k) for k in args.adjoint.split(",")]:
        box = {}

        def rec():
            box["rec"] = api.pn_integrate_record(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"],
                                                 pop["tol"], cap_steps=1024, ckpt_every=K, stream=stream)
        t_rec = _time(rec, args.steps, args.warmup, stream)
        r = box["rec"]
        y = r["y"]
        gy = torch.zeros_like(y)
        gy[1:4] = y[4:7]
        gy[4:7] = y[1:4]
        gy[9] = 1.0
        order = torch.argsort(r["steps"][0], descending=True).to(torch.int32)

        def adj():
            box["g"] = api.pn_integrate_adjoint(d["m"], pop["omega_f"], r, gy, order=order, stream=stream)
        t_adj = _time(adj, args.steps, args.warmup, stream)
        ok = int((r["status"] == 0).sum())
        out["per_K"][K] = {"record_ms": t_rec, "adjoint_ms": t_adj, "r_ckpt": t_rec / t_fwd,
                           "r_bwd": t_adj / t_fwd, "r_total": (t_rec + t_adj) / t_fwd, "ok": ok,
                           "grad_finite": bool(torch.isfinite(box["g"]["S0"]).all())}
    print(json.dumps(out), flush=True)
    return 0


def bench_stats(args, api, w, pop, d, stream) -> int:
    """Time the statistics stage of Sec. V over the workload's own final dot
    products (one JSON line): each operation separately, inputs in HBM."""
    import torch
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], stream=stream)
    y0 = torch.cat([d["omega0"][None], d["S"], d["L"]], 0).contiguous()
    init = api.pn_observables(y0, stream=stream)
    fin = out["dots"]
    torch.cuda.synchronize()
    n = pop["n"]
    sig = api.pn_pearson(init, fin, stream=stream)[:, 3].contiguous()
    ops = {
        "histogram_20": lambda: api.pn_histogram(fin, 20, stream=stream),
        "histogram_100": lambda: api.pn_histogram(fin, 100, stream=stream),
        "histogram2d_79": lambda: api.pn_histogram2d(init, fin, 79, stream=stream),
        "pearson": lambda: api.pn_pearson(init, fin, stream=stream),
        "kde_201": lambda: api.pn_kde(fin, sig, 201, stream=stream),
        "ks_uniform": lambda: api.pn_ks_uniform(fin, stream=stream),
    }
    res = {"metric": "statistics stage (Sec. V) per operation", "workload": w.name, "n": n, "components": 3,
           "ms": {}, "GB_per_s_read": {}}
    reads = {"histogram_20": 24 * n, "histogram_100": 24 * n, "histogram2d_79": 48 * n, "pearson": 96 * n,
             "kde_201": 24 * n, "ks_uniform": 24 * n}
    for k, f in ops.items():
        ms = _time(f, args.steps, args.warmup, stream)
        res["ms"][k] = ms
        res["GB_per_s_read"][k] = reads[k] / (ms * 1e-3) / 1e9
    res["kde_exp_per_s"] = 3 * n * 201 / (res["ms"]["kde_201"] * 1e-3)
    print(json.dumps(res), flush=True)
    return 0


def bench_study(args, api, stream) -> int:
    """The parameter studies of Sec. V B and C on the GPU (one JSON line):
    Pearson r of initial against final dot products against m1 (chi = 1) and
    against chi (m1 = m2), n inspirals per point."""
    import torch
    values = {"m1": [0.5, 0.55, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9],
              "chi": [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0],
              "omega0": [0.002, 0.003, 0.004, 0.005, 0.006, 0.008, 0.01, 0.015, 0.02],
              "omega_f": [0.03, 0.04, 0.05, 0.06, 0.07, 0.08, 0.1]}[args.study]
    # --study-case ring: m1 = 0.4, chi = 0.05 (Sec. V D), for the omega0 and omega_f studies
    fixed = {"m1": 0.4, "chi": 0.05} if args.study_case == "ring" else {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = api.pearson_study(args.study, values, n=args.study_n, stream=stream, **fixed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"metric": f"Pearson r (initial vs final) against {args.study}", "case": args.study_case,
                      "n_per_point": args.study_n,
                      "values": res["values"], "r_S1S2": res["r"][:, 0].tolist(), "r_S1L": res["r"][:, 1].tolist(),
                      "r_S2L": res["r"][:, 2].tolist(), "all_ok": all(res["ok"]), "seconds": dt}), flush=True)
    return 0


def bench_ks_run(args, api, stream) -> int:
    """The K-S test of Sec. V at the paper's size: equal masses, chi_1 = chi_2
    = 0.7, isotropic spins, the Sec. V A frequencies and tolerance
    (omega 0.00395 -> 0.05, tol 5e-7), generated, integrated and tested on the
    GPU in chunks (one JSON line)."""
    import torch
    from paper_0908_3889_amd import population
    w = population.WORKLOADS["paper_equal_mass"]
    spec = api.gen_spec(q=(1.0, 1.0), chi1=(0.7, 0.7), chi2=(0.7, 0.7), omega0=(w.omega0[1], w.omega0[1]),
                        seed=population.BASE_SEED + 12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = api.ks_run(args.ks_run, spec, w.omega_f, w.tol, chunk=1 << 24, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"metric": "K-S test of the final S1_hat.S2_hat against U[-1, 1]", "n": args.ks_run,
                      "D": res["ks"][0].item(), "p": res["ks"][1].item(), "not_ok": int(res["not_ok"]),
                      "hist100": res["hist"].cpu().tolist(), "seconds": dt,
                      "inspirals_per_s": args.ks_run / dt,
                      "setup": "m1 = m2, chi = 0.7, omega 0.00395 -> 0.05, tol 5e-7, Philox seed 9083901"}),
          flush=True)
    return 0


def bench_sweep(args, api, population, stream) -> int:
    """Throughput against the number of inspirals n = 2^8 .. 2^22 (one JSON
    line): n copies of one inspiral (every lane in lock step, the paper's
    Sec. IV set-up) and the first n inspirals of the heterogeneous workload."""
    import torch
    w = population.WORKLOADS[args.workload]
    full = population.generate(w, 2 ** 22)
    rows = []
    for k in range(8, 23, 2):
        n = 2 ** k
        for kind, pop in (("replicated", population.replicate(full, n)),
                          ("heterogeneous", population.subset(full, np.arange(n)))):
            d = api.to_device(pop)
            out = api.alloc_outputs(n)

            def step():
                api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], full["omega_f"], full["tol"],
                                 out=out, stream=stream)
            ms = _time(step, max(2, args.steps // 2), 1, stream)
            ok = bool((out["status"] == 0).all())
            rows.append({"n": n, "kind": kind, "kernel_ms": ms, "inspirals_per_s": n / (ms * 1e-3),
                         "rhs_evals_per_s": float(out["steps"][2].to(torch.int64).sum()) / (ms * 1e-3),
                         "all_ok": ok})
            del d, out
    # the oracle on one host core, on copies of the same inspiral (the
    # paper's CPU figure is one core, Sec. IV)
    import oracle
    one = population.replicate(full, 256)
    t0 = time.perf_counter()
    oracle.integrate(one["m"], one["S"], one["L"], one["omega0"], full["omega_f"], full["tol"], nthreads=1)
    dt = time.perf_counter() - t0
    print(json.dumps({"metric": "throughput vs n", "workload": w.name, "rows": rows,
                      "cpu_baseline": {"value": 256 / dt, "unit": "inspirals/s", "cores": 1, "kind": "oracle",
                                       "sample": "256 copies of inspiral 0"}}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="q1to4_1M")
    ap.add_argument("--schedule", default="persistent", choices=["persistent", "static"])
    ap.add_argument("--order", default="cost", choices=["cost", "natural"],
                    help="hand the inspirals to lanes longest first (pn_cost_order, timed as part of "
                         "every step) or in index order")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--refill-min", type=int, default=0)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32split", "fp32"],
                    help="default: the workload's own precision")
    ap.add_argument("--adjoint", default=None,
                    help="comma-separated checkpoint spacings K: time the recorded forward and the "
                         "discrete adjoint of loss = sum S1.S2 + sum L_hat_z against the plain forward")
    ap.add_argument("--stats", action="store_true",
                    help="time the statistics stage (histograms, Pearson r, KDE, K-S) on the workload's outputs")
    ap.add_argument("--study", default=None, choices=["m1", "chi", "omega0", "omega_f"],
                    help="Pearson r of initial vs final dot products against m1, chi, omega0 or omega_f (Sec. V B, C, D)")
    ap.add_argument("--study-n", type=int, default=65536)
    ap.add_argument("--study-case", default="equal", choices=["equal", "ring"],
                    help="equal: m1 = m2, chi = 1 (Sec. V A set-up); ring: m1 = 0.4, chi = 0.05 (Sec. V D)")
    ap.add_argument("--ks-run", type=int, default=0,
                    help="K-S test of the final S1.S2 over this many inspirals generated on the GPU "
                         "(the paper's run: 362799815)")
    ap.add_argument("--sweep", action="store_true",
                    help="throughput against n = 2^8 .. 2^22, replicated and heterogeneous inspirals")
    ap.add_argument("--calibrate-lanes", action="store_true",
                    help="only run FP64 FMA chains on 64, 32, 16, 4 and 1 active lanes per wave (counter calibration)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three plain device copies of 512 MiB (counter calibration)")
    ap.add_argument("--phase", action="store_true",
                    help="time pn_integrate_phase (the orbital phase integrated alongside)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose refill threshold and block size with pn_autotune on a 2^20 sample first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint, FP32-split and batching legs that follow the timed region")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (--gpus {args.gpus} requested); "
              "the inspirals are independent and would shard by index range across GPUs",
              file=sys.stderr)
        return 2

    import torch

    if args.calibrate_copy:
        return calibrate_copy()
    if args.calibrate_lanes:
        return calibrate_lanes()

    from paper_0908_3889_amd import api, population

    torch.cuda.set_device(0)
    if args.sweep:
        return bench_sweep(args, api, population, torch.cuda.current_stream())
    if args.study:
        return bench_study(args, api, torch.cuda.current_stream())
    if args.ks_run:
        return bench_ks_run(args, api, torch.cuda.current_stream())
    w = population.WORKLOADS[args.workload]
    pop = population.generate(w)
    d = api.to_device(pop)
    out = api.alloc_outputs(pop["n"])
    precision = args.precision or w.precision
    opts = api.make_opts(schedule=args.schedule, block=args.block, precision=precision,
                         waves_per_simd=args.waves_per_simd, refill_min=args.refill_min)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.autotune:
        opts, table = api.autotune(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                                   sample=1 << 20, stream=stream)
        tuned = {"refill_min": opts.refill_min, "block": opts.block,
                 "table_ms": {f"{r},{b}": v for (r, b), v in table.items()}}

    integrate = api.pn_integrate_phase if args.phase else api.pn_integrate
    # the longest-first hand-out order, recomputed inside every timed step
    cost_order = args.order == "cost" and args.schedule == "persistent"
    order_buf = torch.empty((pop["n"],), dtype=torch.int32, device="cuda") if cost_order else None
    order_ws = api.cost_order_workspace(pop["n"]) if cost_order else None
    # the same pass writes the inputs as 128-byte records, which the refills read
    packed_buf = api.packed_inputs(pop["n"]) if cost_order else None
    api.set_order(opts, order_buf)
    api.set_packed(opts, packed_buf)

    def step(kev=None):
        """One pass over the workload; kev: a list that receives the HIP
        events around the integration kernel alone (the dominant kernel)."""
        if cost_order:
            api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], out=order_buf,
                              workspace=order_ws, packed=packed_buf, stream=stream)
        if kev is not None:
            kev.append(torch.cuda.Event(enable_timing=True))
            kev[-1].record(stream)
        integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts, out=out, stream=stream)
        if kev is not None:
            kev.append(torch.cuda.Event(enable_timing=True))
            kev[-1].record(stream)

    if args.adjoint:
        return bench_adjoint(args, api, pop, d, w, step, stream)
    if args.stats:
        return bench_stats(args, api, w, pop, d, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    kev = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step(kev)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    avg_ms = float(np.mean([kev[2 * k].elapsed_time(kev[2 * k + 1]) for k in range(args.steps)]))

    steps = out["steps"].cpu().numpy()
    status = out["status"].cpu().numpy()
    if not (status == 0).all():
        bad = {int(s): int((status == s).sum()) for s in np.unique(status) if s != 0}
        print(f"bench.py: non-OK statuses {bad}", file=sys.stderr)
    flops = algorithmic_flops(steps)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    peak = FP64_VECTOR_PEAK_TFLOPS if precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    n = pop["n"]
    value = n * args.steps / wall
    kernel = (f"integrate_{args.schedule}_{ {'fp64': 'f64', 'fp32split': 'f32s', 'fp32': 'f32x'}[precision] }"
              + ("_phase" if args.phase else ""))
    traffic = measured_traffic(kernel, w.name)
    counter_flop = measured_counter_flop(kernel, w.name)
    resources = kernel_resources(kernel, opts.block or 256)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "inspirals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32split": "f32 stages + f64 state/control",
                  "fp32": "f32 state/stages (compensated omega) + f64 control"}[precision],
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "tol": w.tol, "omega0": list(w.omega0[1:]),
                   "omega_f": w.omega_f, "q": list(w.q[1:]), "chi": list(w.chi[1:]),
                   "precision": precision, "schedule": args.schedule, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "flop_per_unit": {"rhs_evaluation": F_RHS, "attempted_step_besides_rhs": F_STEP_COMB,
                                       "launch": "sum over inspirals of RHS evaluations x F_rhs + "
                                                 "attempted steps x F_comb"},
                     "frac_at_oracle_count": algorithmic_flops(steps, ORACLE_F_RHS, ORACLE_F_STEP_COMB)
                     / (avg_ms * 1e-3) / 1e12 / peak,
                     "frac_at_1300_per_attempted_step": attempted_steps(steps) * PLAN_F_STEP
                     / (avg_ms * 1e-3) / 1e12 / peak,
                     "counter_achieved": (counter_flop / (avg_ms * 1e-3) / 1e12) if counter_flop else None,
                     "counter_frac": (counter_flop / (avg_ms * 1e-3) / 1e12 / peak) if counter_flop else None},
        "kernel": kernel,
        "kernel_resources": resources,
        "launch": {"block": opts.block or 256, "refill_min": opts.refill_min or 4,
                   "waves_per_simd": opts.waves_per_simd or None, "autotuned": tuned},
        "kernel_ms": avg_ms,
        "step_ms_events": step_ms,
        "order": ("cost (pn_cost_order inside every step; the same pass packs the inputs into 128-byte records "
                  "that the refills read)") if cost_order else "natural",
        "rhs_evals_per_s": float(steps[2].astype(np.int64).sum()) / (avg_ms * 1e-3),
        "attempted_steps": attempted_steps(steps),
        "accepted_steps": int(steps[0].astype(np.int64).sum()),
        "rejected_steps": int(steps[1].astype(np.int64).sum()),
        "algorithmic_flop_per_launch": flops,
    }
    if precision != "fp64":
        # the same population in FP64 (untimed) as the reference for the error report
        out64 = integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                          api.make_opts(), stream=stream)
        torch.cuda.synchronize()
        dd = np.abs(out["dots"].cpu().numpy() - out64["dots"].cpu().numpy())
        res["error_vs_fp64"] = {
            "quantity": ["S1h.S2h", "S1h.Lh", "S2h.Lh"],
            "max": dd.max(axis=1).tolist(), "p99": np.percentile(dd, 99, axis=1).tolist(),
            "t_rel_max": float(np.abs(out["t"].cpu().numpy() / out64["t"].cpu().numpy() - 1).max()),
            "reference": "the FP64 GPU path on the whole population (itself within 1e-8 of the oracle)"}
        if args.phase:
            pr = np.abs(out["phase"].cpu().numpy() / out64["phase"].cpu().numpy() - 1)
            res["error_vs_fp64"]["phase_rel_max"] = float(pr.max())
            res["error_vs_fp64"]["phase_rel_p99"] = float(np.percentile(pr, 99))
    # the datasheet peak above, checked on this device (sustained FMA rate)
    res["vector_peak_probe"] = api.pn_fma_rate(8, 4000, stream=stream)
    # the rest of the metric, after the timed region: the adjoint's cost, the
    # FP32-split precision mode and the batching comparison
    if not args.no_extras and w.name == "q1to4_1M" and precision == "fp64" and not args.phase:
        ref64 = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        res["adjoint"] = leg_adjoint(api, population, stream)
        res["fp32split"] = leg_fp32split(api, pop, d, ref64, stream)
        res["fp32_state"] = leg_fp32split(api, pop, d, ref64, stream, precision="fp32")
        res["batching"] = leg_batching(api, population, stream)
        res["cpu_check"] = leg_check(api, pop, d, stream)
    if not args.no_cpu_baseline:
        gpu = {"dots": out["dots"].cpu().numpy(), "steps": steps, "status": status}
        # FP32-split is checked against the FP64 oracle with its own error bound
        res["cpu_baseline"] = cpu_baseline(pop, args.cpu_budget, gpu, 1e-8 if precision == "fp64" else 1e-3)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
