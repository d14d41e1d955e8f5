"""The FP32-split arithmetic mode against the FP64 oracle.

FP32-split evaluates the stages and right-hand sides in single precision
(the paper's GPU arithmetic, Sec. III) and keeps the state, t, h, the error
norm, the step control and the omega_f test in double.  It is not expected
to reproduce the FP64 step sequence; it is expected to land on omega_f with
final dot products within the accuracy that FP32 right-hand sides allow.
The bounds below are the measured error plus margin; the measured values
are printed (and reported by bench.py for the full population)."""
import numpy as np
import pytest

from helpers import normwise_rel, run_gpu, run_oracle
from paper_0908_3889_amd import population as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3889_amd import _lib
    _lib.load()
    yield


def _errors(rg, ro):
    d = np.abs(rg["dots"] - ro["dots"])
    return d.max(axis=1), np.percentile(d, 99, axis=1)


@pytest.mark.parametrize("workload,n,max_bound,p99_bound", [
    ("q1to4_1M", 4099, 2e-4, 5e-5), ("equal_mass_maxspin_1k", 1024, 2e-4, 5e-5),
    ("batching_4M", 2049, 1e-3, 2e-4), ("adjoint_64k", 1000, 2e-4, 5e-5)])
def test_fp32split_dots_against_fp64_oracle(workload, n, max_bound, p99_bound):
    pop = P.generate(workload, n)
    if workload == "equal_mass_maxspin_1k":
        pop["tol"] = 1e-8          # FP32 stages cannot resolve 1e-10
    ro = run_oracle(pop)
    rg = run_gpu(pop, precision="fp32split")
    assert (rg["status"] == 0).all() and (ro["status"] == 0).all()
    assert (rg["y"][0] == pop["omega_f"]).all()
    mx, p99 = _errors(rg, ro)
    print(f"{workload}: max |dots - oracle| = {mx}, p99 = {p99}")
    assert (mx < max_bound).all(), mx
    assert (p99 < p99_bound).all(), p99
    assert np.abs(rg["t"] / ro["t"] - 1).max() < 1e-5


def test_fp32split_fixed_step_against_fp64_oracle():
    pop = P.generate("adjoint_64k", 500)
    ro = run_oracle(pop, h_fixed=50.0)
    rg = run_gpu(pop, h_fixed=50.0, precision="fp32split")
    assert (rg["status"] == 0).all()
    np.testing.assert_array_equal(rg["steps"][:2], ro["steps"][:2])
    err = normwise_rel(rg["y"], ro["y"], pop["S"])
    print("fixed-step FP32-split normwise error: max", err.max(), "median", np.median(err))
    assert err.max() < 1e-4


def test_fp32split_launch_shapes_agree_bitwise():
    pop = P.generate("batching_4M", 1500)
    base = run_gpu(pop, precision="fp32split")
    for kw in (dict(schedule="static"), dict(block=64), dict(waves_per_simd=1), dict(refill_min=1), dict(refill_min=16)):
        other = run_gpu(pop, precision="fp32split", **kw)
        for k in ("y", "t", "steps", "status", "dots"):
            np.testing.assert_array_equal(other[k], base[k], err_msg=f"{kw} {k}")


def test_fp32split_status_codes():
    pop = P.generate("q1to4_1M", 70)
    pop["omega0"] = pop["omega0"].copy(); pop["m"] = pop["m"].copy()
    pop["omega0"][0] = 0.06
    pop["m"][1, 2] = 0.0
    rg = run_gpu(pop, precision="fp32split")
    assert rg["status"][0] == 1 and rg["status"][2] == -4
    assert (rg["status"][3:] == 0).all()
    r2 = run_gpu(pop, precision="fp32split", max_steps=5)
    assert (r2["status"][3:] == -1).all()


def test_fp32split_full_size_samples():
    """The whole 1M population in FP32-split, in the benchmark's launch
    configuration, checked on 512 sampled inspirals against the FP64 oracle
    with the bounds above."""
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M")
    d = api.to_device(pop)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                           api.make_opts(precision="fp32split"))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert (st == 0).all()
    assert bool((out["y"][0] == pop["omega_f"]).all())
    idx = np.sort(np.random.default_rng(31).choice(st.size, 512, replace=False))
    ro = run_oracle(P.subset(pop, idx))
    dots = out["dots"].cpu().numpy()[:, idx]
    d_err = np.abs(dots - ro["dots"])
    print("FP32-split full size, 512 samples: max", d_err.max(axis=1), "p99", np.percentile(d_err, 99, axis=1))
    assert (d_err.max(axis=1) < 2e-4).all() and (np.percentile(d_err, 99, axis=1) < 5e-5).all()
    t = out["t"].cpu().numpy()[idx]
    assert np.abs(t / ro["t"] - 1).max() < 1e-5
