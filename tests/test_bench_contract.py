"""bench.py's output contract: the JSON line's fields, the CPU baseline leg,
the HBM-traffic lookup, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_0908_3889_amd import population as P  # noqa: E402

REQUIRED = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "roofline"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields():
    pop = P.generate("equal_mass_maxspin_1k", 64)
    cb = bench.cpu_baseline(pop, budget_s=0.1)
    assert cb["kind"] == "oracle" and cb["unit"] == "inspirals/s"
    assert cb["value"] > 0 and cb["cores"] == len(os.sched_getaffinity(0))
    assert cb["sample"].startswith("first ") and "of 64 inspirals of equal_mass_maxspin_1k" in cb["sample"]
    assert cb["rhs_evals_per_s"] > cb["value"]
    assert cb["per_core"]["value"] > 0 and "one thread" in cb["per_core"]["sample"]


def test_algorithmic_flops_from_step_counts():
    steps = np.array([[10, 20], [2, 0], [1 + 6 * 12, 1 + 6 * 20]], dtype=np.int32)
    attempted = np.array([12, 20])
    want = (steps[2].astype(np.int64) * bench.F_RHS).sum() + (attempted * bench.F_STEP_COMB).sum()
    assert bench.algorithmic_flops(steps) == float(want)


def test_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    from paper_0908_3889_amd import build
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("integrate_persistent_f64", "q1to4_1M") is None     # no summary
    f = tmp_path / "hbm_integrate_persistent_f64_q1to4_1M.txt"
    f.write_text(f"# x\nhbm_bytes_per_launch: 123456\nsource_digest: {build.source_digest()}\n")
    assert bench.measured_traffic("integrate_persistent_f64", "q1to4_1M") == 123456.0
    f.write_text("# x\nhbm_bytes_per_launch: 123456\nsource_digest: 0000\n")
    assert bench.measured_traffic("integrate_persistent_f64", "q1to4_1M") is None     # stale


@pytest.mark.gpu
def test_bench_line_on_the_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "equal_mass_maxspin_1k",
                        "--steps", "2", "--warmup", "1", "--no-cpu-baseline"], capture_output=True, text=True,
                       cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    res = json.loads(lines[0])
    assert REQUIRED <= set(res)
    assert res["n_gpus"] == 1 and res["steps"] == 2 and res["warmup"] == 1
    assert res["value"] > 0 and res["ms_per_step"] > 0 and res["higher_is_better"] is True
    assert res["vs_baseline"] is None and res["data"] == "synthetic" and res["dtype"] == "f64"
    assert res["config"]["workload"] == "equal_mass_maxspin_1k" and res["config"]["n"] == 1024
    rf = res["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert 0 < rf["frac"] < 1 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert res["kernel"] == "integrate_persistent_f64"
    assert res["accepted_steps"] > 0 and res["kernel_ms"] > 0
    # the probe of the vector peak: FP32 without packed instructions and FP64
    # both issue one wave64 FMA per four cycles per SIMD, the 78.6 TFLOP/s of
    # the datasheet's FP64 figure (256 CUs x 2.4 GHz x 128 FLOP/clock)
    pk = res["vector_peak_probe"]
    for k in ("fp32_nonpacked", "fp64"):
        assert 0.6 * 78.6 < pk[k] < 1.02 * 78.6, pk


@pytest.mark.gpu
def test_bench_legs_on_the_gpu():
    """The adjoint, FP32-split and batching legs of the default line, on small
    prefixes of their workloads."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3889_amd import api
    stream = torch.cuda.current_stream()
    adj = bench.leg_adjoint(api, P, stream, ks=(16, 64), reps=2, n=2048)
    assert adj["n"] == 2048 and set(adj["per_K"]) == {"16", "64"}
    for v in adj["per_K"].values():
        assert v["ok"] == 2048 and v["grad_finite"] and v["r_bwd"] > 0 and v["r_ckpt"] > 0
        assert abs(v["r_bwd"] - v["adjoint_ms"] / adj["fwd_ms"]) < 1e-12
    pop = P.generate("q1to4_1M", 8192)
    d = api.to_device(pop)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], stream=stream)
    ref64 = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    f32 = bench.leg_fp32split(api, pop, d, ref64, stream, reps=2)
    assert f32["status_ok"] == 8192 and 0 < f32["frac"] < 1
    e = f32["error_vs_fp64"]
    assert set(e) == {"S1h.S2h", "S1h.Lh", "S2h.Lh", "S1 (|dS1|/|S1(0)|)", "S2 (|dS2|/|S2(0)|)", "L_hat (|dL|)",
                      "t (relative)", "phase (relative)"}
    assert all(0 <= v["p99"] <= v["max"] < 1e-2 for v in e.values())
    bat = bench.leg_batching(api, P, stream, reps=1, n=16384)
    assert bat["persistent"]["status_ok"] == 16384 and bat["static"]["status_ok"] == 16384
    assert bat["static_over_persistent"] > 0


@pytest.mark.gpu
def test_bench_cpu_baseline_and_crosscheck_on_the_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "equal_mass_maxspin_1k",
                        "--steps", "2", "--warmup", "1", "--cpu-budget", "1"], capture_output=True, text=True,
                       cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    cb = json.loads(r.stdout.strip().splitlines()[-1])["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0
    cc = cb["crosscheck"]
    assert cc["ok"] and cc["n"] > 0 and cc["status_mismatches"] == 0 and cc["step_count_mismatches"] == 0
    assert cc["max_dot_diff"] < 1e-8


def test_cpu_baseline_crosscheck_flags_disagreement():
    import oracle
    pop = P.generate("equal_mass_maxspin_1k", 48)
    r = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"])
    gpu = {"dots": oracle.observables(r["y"]), "steps": r["steps"].astype(np.int32), "status": r["status"]}
    cc = bench.cpu_baseline(pop, budget_s=0.05, gpu=gpu)["crosscheck"]
    assert cc["ok"] and cc["n"] == 48 and cc["max_dot_diff"] == 0.0
    assert cc["status_mismatches"] == 0 and cc["step_count_mismatches"] == 0
    bad = {k: v.copy() for k, v in gpu.items()}
    bad["dots"][1, 5] += 1e-6
    bad["steps"][0, 7] += 1
    cc = bench.cpu_baseline(pop, budget_s=0.05, gpu=bad)["crosscheck"]
    assert not cc["ok"] and abs(cc["max_dot_diff"] - 1e-6) < 1e-12 and cc["step_count_mismatches"] == 1
    bad = {k: v.copy() for k, v in gpu.items()}
    bad["status"][3] = -1
    cc = bench.cpu_baseline(pop, budget_s=0.05, gpu=bad)["crosscheck"]
    assert not cc["ok"] and cc["status_mismatches"] == 1
