"""The host integrator of the CPU check (pn_check_integrate_host, product
code in csrc/pn_check.cpp) against the oracle.  Both are FP64
implementations of the same method, so the step sequences must agree and
the final states must agree to rounding; and the comparison step of
pn_check_finish must flag exactly the inspirals whose outputs were
disturbed.  These tests need no GPU: the library runs them on the host."""
import ctypes as C

import numpy as np
import pytest

from helpers import normwise_rel, run_oracle
from paper_0908_3889_amd import population as P


@pytest.fixture(scope="module")
def api():
    from paper_0908_3889_amd import _lib, api
    try:
        _lib.load()
    except _lib.PnError as e:
        pytest.skip(str(e))
    return api


def _host(api, pop, **kw):
    opts = api.make_opts(**kw)
    return api.check_integrate_host(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"], opts)


@pytest.mark.parametrize("workload,n", [("equal_mass_maxspin_1k", 256), ("q1to4_1M", 512),
                                        ("batching_4M", 256), ("adjoint_64k", 256)])
def test_adaptive_host_integrator_against_oracle(api, workload, n):
    pop = P.generate(workload, n)
    rh = _host(api, pop)
    ro = run_oracle(pop)
    np.testing.assert_array_equal(rh["status"], ro["status"])
    np.testing.assert_array_equal(rh["steps"], ro["steps"])
    ok = ro["status"] == 0
    assert (rh["y"][0][ok] == pop["omega_f"]).all()
    err = normwise_rel(rh["y"], ro["y"], pop["S"])[ok]
    dots = api_dots(rh["y"])
    d_err = np.abs(dots - ro["dots"])[:, ok]
    print(f"{workload}: normwise max {err.max():.3e}, dots max {d_err.max():.3e}, "
          f"t max rel {np.abs(rh['t'] / ro['t'] - 1)[ok].max():.3e}")
    assert d_err.max() < 1e-11
    assert err.max() < 1e-10
    assert np.abs(rh["t"] / ro["t"] - 1)[ok].max() < 1e-10


def api_dots(y):
    """Unit dot products of final states (0 where a norm is 0)."""
    n1 = np.linalg.norm(y[1:4], axis=0); n2 = np.linalg.norm(y[4:7], axis=0); nl = np.linalg.norm(y[7:10], axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.stack([(y[1:4] * y[4:7]).sum(0) / (n1 * n2), (y[1:4] * y[7:10]).sum(0) / (n1 * nl),
                      (y[4:7] * y[7:10]).sum(0) / (n2 * nl)])
    return np.nan_to_num(d)


@pytest.mark.parametrize("workload,h", [("equal_mass_maxspin_1k", 40.0), ("q1to4_1M", 100.0)])
def test_fixed_step_host_integrator_against_oracle(api, workload, h):
    pop = P.generate(workload, 128)
    rh = _host(api, pop, h_fixed=h)
    ro = run_oracle(pop, h_fixed=h)
    np.testing.assert_array_equal(rh["steps"][:2], ro["steps"][:2])
    err = normwise_rel(rh["y"], ro["y"], pop["S"])
    print(f"fixed-step {workload}: normwise max {err.max():.3e}")
    assert err.max() < 1e-12


def test_t_end_and_term_switches_against_oracle(api):
    pop = P.generate("adjoint_64k", 64)
    for kw in (dict(t_end=12000.0), dict(terms=1 | 8), dict(theta_literal=1)):
        rh = _host(api, pop, **kw)
        ro = run_oracle(pop, **kw)
        np.testing.assert_array_equal(rh["steps"][:2], ro["steps"][:2])
        np.testing.assert_array_equal(rh["status"], ro["status"])
        assert normwise_rel(rh["y"], ro["y"], pop["S"]).max() < 1e-10, kw


def test_statuses_against_oracle(api):
    pop = P.generate("q1to4_1M", 40)
    pop["omega0"][0] = 0.06                 # done at start
    pop["m"][1, 2] = 0.0                    # bad input
    pop["S"][0, 3] = np.nan                 # bad input
    rh = _host(api, pop)
    ro = run_oracle(pop)
    np.testing.assert_array_equal(rh["status"], ro["status"])
    assert rh["status"][0] == 1 and rh["status"][2] == -4 and rh["status"][3] == -4
    r5 = _host(api, pop, max_steps=5)
    o5 = run_oracle(pop, max_steps=5)
    np.testing.assert_array_equal(r5["status"], o5["status"])
    np.testing.assert_array_equal(r5["steps"][:2], o5["steps"][:2])


def test_threads_do_not_change_results(api):
    pop = P.generate("batching_4M", 300)
    opts = api.make_opts()
    a = api.check_integrate_host(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"], opts, 1)
    b = api.check_integrate_host(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"], opts, 5)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_finish_flags_exactly_the_disturbed_inspirals(api):
    """pn_check_start / pn_check_finish on host arrays: the 'GPU' outputs
    here are the oracle's (equal to the host integrator's to rounding), with
    planted disagreements."""
    from paper_0908_3889_amd import _lib
    L = _lib.load()
    pop = P.generate("adjoint_64k", 50)
    ro = run_oracle(pop)
    y = np.ascontiguousarray(ro["y"].copy())
    steps = np.ascontiguousarray(ro["steps"].astype(np.int32))
    status = np.ascontiguousarray(ro["status"].astype(np.int32))
    y[1:4, 7] = y[1:4, 7][::-1].copy()       # a different spin direction: dot products change
    status[11] = -3                          # a different status
    steps[0, 20] += 1                        # a different step count: counted, not flagged
    y[2, 30] += 1e-12                        # within the bar: not flagged
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    o = _lib.PnOpts()
    assert L.pn_check_start(C.byref(h), 50, 50, p(pop["m"]), p(pop["S"]), p(pop["L"]), p(pop["omega0"]),
                            pop["omega_f"], pop["tol"], C.byref(o), 3) == 0
    flags = np.full(50, -1, dtype=np.int32)
    rep = _lib.PnCheckReport()
    assert L.pn_check_finish(h, p(y), p(steps), p(status), 50, 1e-8, p(flags), C.byref(rep)) == 0
    assert rep.checked == 50 and rep.flagged == 2 and rep.status_mismatches == 1 and rep.step_mismatches == 1
    assert flags[7] == 2 and flags[11] == 1
    assert (np.delete(flags, [7, 11]) == 0).all()
    assert rep.max_dot_diff > 1e-3 and rep.host_seconds > 0


def test_check_argument_errors(api):
    from paper_0908_3889_amd import _lib
    L = _lib.load()
    h = C.c_void_p()
    z = C.c_void_p(0)
    o = _lib.PnOpts()
    assert L.pn_check_start(None, 1, 1, z, z, z, z, 0.05, 1e-8, C.byref(o), 1) == _lib.PN_EINVAL
    assert L.pn_check_start(C.byref(h), 5, 4, z, z, z, z, 0.05, 1e-8, C.byref(o), 1) == _lib.PN_EINVAL
    assert L.pn_check_start(C.byref(h), 5, 5, z, z, z, z, 0.05, 1e-8, C.byref(o), 1) == _lib.PN_EINVAL
    assert L.pn_check_finish(None, z, z, z, 0, 1e-8, z, None) == _lib.PN_EINVAL
    # an empty sample starts and finishes
    assert L.pn_check_start(C.byref(h), 0, 0, z, z, z, z, 0.05, 1e-8, C.byref(o), 1) == 0
    rep = _lib.PnCheckReport()
    assert L.pn_check_finish(h, z, z, z, 0, 1e-8, z, C.byref(rep)) == 0 and rep.checked == 0
    assert L.pn_check_integrate_host(3, 2, z, z, z, z, 0.05, 1e-8, C.byref(o), z, z, z, z, 1) == _lib.PN_EINVAL
