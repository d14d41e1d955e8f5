"""The FP32 arithmetic modes against the FP64 oracle.

FP32-split evaluates the stages and right-hand sides in single precision
(the paper's GPU arithmetic, Sec. III) and keeps the state, t, h, the error
norm, the step control and the omega_f test in double.  FP32-state
(precision "fp32") holds the state in single precision too, with omega and
the phase as compensated sums.  Neither is expected to reproduce the FP64
step sequence; each is expected to land on omega_f with final dot products,
spins, L_hat and t within the accuracy its arithmetic allows.  The bounds
below are the measured error plus margin; the measured values are printed
(and reported by bench.py for the full population)."""
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


PRECISIONS = ("fp32split", "fp32")
# error bounds per mode (max, p99): dot products; S1, S2 (relative to
# |S_i(0)|) and L_hat; the FP32 state adds its own rounding, about three
# times the FP32-split error
BOUNDS = {"fp32split": {"dots": (2e-4, 5e-5), "vec": (1e-3, 2e-5)},
          "fp32": {"dots": (1e-3, 1e-4), "vec": (3e-3, 1e-4)}}


def _errors(rg, ro):
    d = np.abs(rg["dots"] - ro["dots"])
    return d.max(axis=1), np.percentile(d, 99, axis=1)


def _vector_errors(rg, ro, S0):
    """max and p99 of |S1 - S1_oracle|/|S1(0)|, the same for S2, and |L - L_oracle|."""
    n1 = np.linalg.norm(S0[:3], axis=0); n1[n1 == 0] = 1.0
    n2 = np.linalg.norm(S0[3:], axis=0); n2[n2 == 0] = 1.0
    e = {"S1": np.linalg.norm(rg["y"][1:4] - ro["y"][1:4], axis=0) / n1,
         "S2": np.linalg.norm(rg["y"][4:7] - ro["y"][4:7], axis=0) / n2,
         "L_hat": np.linalg.norm(rg["y"][7:10] - ro["y"][7:10], axis=0)}
    return {k: (float(v.max()), float(np.percentile(v, 99))) for k, v in e.items()}


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("workload,n,scale", [
    ("q1to4_1M", 4099, 1.0), ("equal_mass_maxspin_1k", 1024, 1.0),
    ("batching_4M", 2049, 5.0), ("adjoint_64k", 1000, 1.0)])
def test_fp32_dots_and_state_against_fp64_oracle(workload, n, scale, precision):
    pop = P.generate(workload, n)
    if workload == "equal_mass_maxspin_1k":
        pop["tol"] = 1e-8          # FP32 stages cannot resolve 1e-10
    ro = run_oracle(pop)
    rg = run_gpu(pop, precision=precision)
    assert (rg["status"] == 0).all() and (ro["status"] == 0).all()
    assert (rg["y"][0] == pop["omega_f"]).all()
    mx, p99 = _errors(rg, ro)
    vec = _vector_errors(rg, ro, pop["S"])
    t_rel = np.abs(rg["t"] / ro["t"] - 1)
    print(f"{workload} {precision}: max |dots - oracle| = {mx}, p99 = {p99}; "
          f"S1, S2, L_hat (max, p99) = {vec}; t relative max {t_rel.max():.3e} p99 {np.percentile(t_rel, 99):.3e}")
    dmax, dp99 = BOUNDS[precision]["dots"]
    assert (mx < dmax * scale).all(), mx
    assert (p99 < dp99 * scale).all(), p99
    vmax, vp99 = BOUNDS[precision]["vec"]
    for k, (a, b) in vec.items():
        assert a < vmax * scale and b < vp99 * scale, (k, a, b)
    assert t_rel.max() < 1e-5


@pytest.mark.parametrize("precision", PRECISIONS)
def test_fp32_fixed_step_against_fp64_oracle(precision):
    pop = P.generate("adjoint_64k", 500)
    ro = run_oracle(pop, h_fixed=50.0)
    rg = run_gpu(pop, h_fixed=50.0, precision=precision)
    assert (rg["status"] == 0).all()
    np.testing.assert_array_equal(rg["steps"][:2], ro["steps"][:2])
    err = normwise_rel(rg["y"], ro["y"], pop["S"])
    print(f"fixed-step {precision} normwise error: max", err.max(), "median", np.median(err))
    assert err.max() < 1e-4


@pytest.mark.parametrize("precision", PRECISIONS)
def test_fp32_launch_shapes_agree_bitwise(precision):
    pop = P.generate("batching_4M", 1500)
    base = run_gpu(pop, precision=precision)
    for kw in (dict(schedule="static"), dict(block=64), dict(waves_per_simd=1), dict(refill_min=1), dict(refill_min=16)):
        other = run_gpu(pop, precision=precision, **kw)
        for k in ("y", "t", "steps", "status", "dots"):
            np.testing.assert_array_equal(other[k], base[k], err_msg=f"{kw} {k}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_fp32_status_codes(precision):
    pop = P.generate("q1to4_1M", 70)
    pop["omega0"] = pop["omega0"].copy(); pop["m"] = pop["m"].copy()
    pop["omega0"][0] = 0.06
    pop["m"][1, 2] = 0.0
    rg = run_gpu(pop, precision=precision)
    assert rg["status"][0] == 1 and rg["status"][2] == -4
    assert (rg["status"][3:] == 0).all()
    r2 = run_gpu(pop, precision=precision, max_steps=5)
    assert (r2["status"][3:] == -1).all()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_fp32_full_size_samples(precision):
    """The whole 1M population, in the benchmark's launch configuration,
    checked on 512 sampled inspirals against the FP64 oracle with the bounds
    above."""
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M")
    d = api.to_device(pop)
    order = api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"])
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                           api.make_opts(precision=precision, order=order))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert (st == 0).all()
    assert bool((out["y"][0] == pop["omega_f"]).all())
    idx = np.sort(np.random.default_rng(31).choice(st.size, 512, replace=False))
    ro = run_oracle(P.subset(pop, idx))
    g = {k: v.cpu().numpy()[..., idx] for k, v in out.items() if v is not None}
    d_err = np.abs(g["dots"] - ro["dots"])
    vec = _vector_errors(g, ro, pop["S"][:, idx])
    print(f"{precision} full size, 512 samples: max", d_err.max(axis=1), "p99", np.percentile(d_err, 99, axis=1),
          "S1, S2, L_hat (max, p99)", vec)
    dmax, dp99 = BOUNDS[precision]["dots"]
    assert (d_err.max(axis=1) < dmax).all() and (np.percentile(d_err, 99, axis=1) < dp99).all()
    assert np.abs(g["t"] / ro["t"] - 1).max() < 1e-5
