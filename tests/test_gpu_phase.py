"""pn_integrate_phase (the orbital phase, d Phi/dt = omega) on the GPU against
the oracle's phase, and against pn_integrate.

The phase is outside the error norm, so every other output must be
bit-identical to pn_integrate's.  FP64: fixed steps to 1e-12 relative (1e-15
per step on long runs, as for the state), adaptive runs to 1e-9 relative
with identical step counts (as for t_final).  FP32-split: the phase is
summed in FP64 from FP32 increments; the bound is the measured error plus
margin, as for the other FP32-split outputs, and the measured error is
printed."""
import numpy as np
import pytest

import oracle
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


def _api():
    from paper_0908_3889_amd import api
    return api


def _run(pop, phase, **kw):
    api = _api()
    d = api.to_device(pop)
    fn = api.pn_integrate_phase if phase else api.pn_integrate
    out = fn(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], api.make_opts(**kw))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _oracle(pop, **kw):
    return oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"], phase=True,
                            **kw)


@pytest.mark.parametrize("kw", [dict(), dict(precision="fp32split"), dict(schedule="static"),
                                dict(block=64, refill_min=1), dict(precision="fp32split", schedule="static"),
                                dict(precision="fp32"), dict(precision="fp32", schedule="static"),
                                dict(h_fixed=80.0), dict(t_end=3.0e4)])
def test_other_outputs_bit_identical_to_pn_integrate(kw):
    pop = P.generate("batching_4M", 3001)
    a = _run(pop, False, **kw)
    b = _run(pop, True, **kw)
    for k in ("y", "t", "steps", "status", "dots"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{kw} {k}")
    assert np.isfinite(b["phase"]).all() and (b["phase"][b["status"] == 0] > 0).all()


@pytest.mark.parametrize("workload,h", [("equal_mass_maxspin_1k", 40.0), ("q1to4_1M", 100.0),
                                        ("batching_4M", 100.0)])
def test_fixed_step_phase_parity(workload, h):
    pop = P.generate(workload, 777)
    ro = _oracle(pop, h_fixed=h)
    rg = _run(pop, True, h_fixed=h)
    assert (rg["status"] == ro["status"]).all()
    np.testing.assert_array_equal(rg["steps"][:2], ro["steps"][:2])
    bound = 1e-12
    rel = np.abs(rg["phase"] / ro["phase"] - 1)
    steps = ro["steps"][0]
    print(f"\nfixed-step phase {workload} h={h}: max rel {rel.max():.3e}, median {np.median(rel):.3e}, "
          f"max rel/step {(rel / steps).max():.3e}, max rel/sqrt(step) {(rel / np.sqrt(steps)).max():.3e}, "
          f"steps {steps.min()}..{steps.max()}", flush=True)
    assert (rel < bound).all(), (rel / bound).max()


@pytest.mark.parametrize("workload,n", [("equal_mass_maxspin_1k", 1024), ("q1to4_1M", 4099),
                                        ("batching_4M", 2049), ("paper_timing", 300)])
def test_adaptive_phase_parity(workload, n):
    pop = P.generate(workload, n)
    ro = _oracle(pop)
    rg = _run(pop, True)
    assert (rg["status"] == ro["status"]).all()
    np.testing.assert_array_equal(rg["steps"][:2], ro["steps"][:2])
    ok = ro["status"] == 0
    rel = np.abs(rg["phase"] / ro["phase"] - 1)[ok]
    assert rel.max() < 1e-9, rel.max()


def test_adaptive_t_end_phase_parity():
    pop = P.generate("adjoint_64k", 500)
    ro = _oracle(pop, t_end=12000.0)
    rg = _run(pop, True, t_end=12000.0)
    np.testing.assert_array_equal(rg["steps"][:2], ro["steps"][:2])
    assert np.abs(rg["phase"] / ro["phase"] - 1).max() < 1e-9


@pytest.mark.parametrize("precision", ["fp32split", "fp32"])
def test_fp32_phase_against_fp64_oracle(precision):
    pop = P.generate("q1to4_1M", 4099)
    ro = _oracle(pop)
    rg = _run(pop, True, precision=precision)
    assert (rg["status"] == 0).all()
    rel = np.abs(rg["phase"] / ro["phase"] - 1)
    print(f"{precision} phase: max rel error {rel.max():.3e}, p99 {np.percentile(rel, 99):.3e}, "
          f"max abs {np.abs(rg['phase'] - ro['phase']).max():.3e} rad")
    # FP32-split measured 1.0e-7 max and 7e-8 p99 on these inspirals (1.2e-7 /
    # 7e-8 over the whole 1M population): the FP32 rounding of each step's
    # increment, summed in FP64 without further growth; the FP32 state sums
    # the increments with their rounding errors (compensated)
    assert rel.max() < 1e-6 and np.percentile(rel, 99) < 5e-7


def test_phase_of_special_statuses_and_sizes():
    api = _api()
    pop = P.generate("adjoint_64k", 70)
    pop["omega0"][3] = 0.07                      # DONE_AT_START
    pop["m"][0, 5] = np.nan                      # BAD_INPUT
    ro = _oracle(pop)
    rg = _run(pop, True)
    assert rg["status"][3] == 1 and rg["status"][5] == -4
    assert rg["phase"][3] == 0.0 and rg["phase"][5] == 0.0
    ok = ro["status"] == 0
    assert np.abs(rg["phase"][ok] / ro["phase"][ok] - 1).max() < 1e-9
    # n = 0 launches nothing; n = 1 is one lane of one wave
    d = api.to_device(P.generate("adjoint_64k", 1))
    out = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], 0.05, 1e-8)
    one = _oracle(P.generate("adjoint_64k", 1))
    assert abs(out["phase"].item() / one["phase"][0] - 1) < 1e-9
    e = {k: v[..., :0] for k, v in d.items()}
    out = api.pn_integrate_phase(e["m"], e["S"], e["L"], e["omega0"], 0.05, 1e-8)
    assert out["phase"].numel() == 0


def test_full_size_phase_samples():
    """The 1M workload in the launch configuration the benchmark times, checked
    on a sample of 256 inspirals that the oracle integrates one by one."""
    api = _api()
    pop = P.generate("q1to4_1M")
    d = api.to_device(pop)
    out = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    torch.cuda.synchronize()
    idx = np.random.default_rng(7).choice(pop["omega0"].size, 256, replace=False)
    sub = P.subset(pop, idx)
    ro = _oracle(sub)
    ph = out["phase"].cpu().numpy()[idx]
    st = out["status"].cpu().numpy()[idx]
    steps = out["steps"].cpu().numpy()[:, idx]
    assert (st == 0).all()
    np.testing.assert_array_equal(steps[:2], ro["steps"][:2])
    assert np.abs(ph / ro["phase"] - 1).max() < 1e-9
