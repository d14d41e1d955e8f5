"""The oracle's orbital phase Phi (d Phi/dt = omega, Phi(0) = 0) against what
fixes it independently of the integrator: the Newtonian closed forms, the
constant-frequency case, quadrature for aligned spins, the convergence order
of the fixed-step scheme, the symmetries of the problem, and the step
sequence, which must not change when the phase is integrated alongside.

The phase is not a quantity of the paper; it is the added output of the
waveform-style studies (the integral of the orbital frequency)."""
import numpy as np
import pytest
from scipy import integrate as si

import oracle

NT = 8


def _one(m1, m2, S1, S2, L, w0):
    return (np.array([[m1], [m2]]), np.concatenate([S1, S2]).reshape(6, 1),
            np.asarray(L, float).reshape(3, 1), np.array([w0]))


def _random_pop(n, seed, q=(1, 4), chi=(0.3, 1.0), w0=0.005):
    rng = np.random.default_rng(seed)
    qq = rng.uniform(*q, n)
    m1, m2 = qq / (1 + qq), 1 / (1 + qq)
    u = rng.normal(size=(3, 3, n))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    c1, c2 = rng.uniform(*chi, n), rng.uniform(*chi, n)
    return np.stack([m1, m2]), np.concatenate([c1 * m1 ** 2 * u[0], c2 * m2 ** 2 * u[1]]), u[2], np.full(n, w0)


def _newtonian(q):
    m1, m2 = q / (1 + q), 1 / (1 + q)
    eta = m1 * m2
    z = np.zeros(3)
    return (m1, m2, z, z, [0.0, 0.0, 1.0]), eta


@pytest.mark.parametrize("q,w0,wf", [(1.0, 0.005, 0.05), (4.0, 0.01, 0.05), (10.0, 0.002, 0.1)])
def test_newtonian_phase_to_omega_f(q, w0, wf):
    """Leading order: d omega/dt = (96/5) eta M^{5/3} omega^{11/3}, so
    d Phi/d omega = omega / omega-dot integrates to
    Phi* = (w0^{-5/3} - wf^{-5/3}) / (32 eta M^{5/3})."""
    args, eta = _newtonian(q)
    m, S, L, w = _one(*args, w0)
    exact = (w0 ** (-5 / 3) - wf ** (-5 / 3)) / (32 * eta)
    errs = []
    for tol in (1e-10, 1e-11, 1e-12, 1e-13):
        r = oracle.integrate(m, S, L, w, wf, tol, terms=oracle.TERM_RR, phase=True)
        assert r["status"][0] == 0
        errs.append(abs(r["phase"][0] / exact - 1))
    assert errs[-1] < 1e-10, errs
    assert all(errs[k + 1] < errs[k] / 5 for k in range(3)), errs


@pytest.mark.parametrize("frac", [0.3, 0.9, 0.999])
def test_newtonian_phase_at_time(frac):
    """Phi(t) = (w0^{-5/3} - omega(t)^{-5/3}) / (32 eta M^{5/3}) with the
    closed-form omega(t) = [w0^{-8/3} - (256/5) eta M^{5/3} t]^{-3/8}."""
    q, w0 = 2.0, 0.004
    args, eta = _newtonian(q)
    m, S, L, w = _one(*args, w0)
    tc = w0 ** (-8 / 3) / (256 / 5 * eta)
    t_end = frac * tc
    om = (w0 ** (-8 / 3) - 256 / 5 * eta * t_end) ** (-3 / 8)
    exact = (w0 ** (-5 / 3) - om ** (-5 / 3)) / (32 * eta)
    errs = []
    for tol in (1e-11, 1e-12, 1e-13, 1e-14):
        r = oracle.integrate(m, S, L, w, 0.1, tol, terms=oracle.TERM_RR, t_end=t_end, phase=True)
        assert r["status"][0] == 0
        errs.append(abs(r["phase"][0] / exact - 1))
    # the signed error can cross zero between two tolerances, so the
    # convergence is checked over the three decades as a whole
    assert errs[-1] < 1e-11, errs
    assert errs[-1] < errs[0] / 100, errs


def test_constant_frequency_phase_is_omega_times_t():
    """Without radiation reaction omega is constant and Phi = omega0 t: every
    stage value of omega is omega0 and the weights sum to 1, so the result is
    exact up to the rounding of the weighted sums."""
    m, S, L, w = _random_pop(16, 3, w0=0.02)
    w = w * np.linspace(0.5, 2.0, 16)
    for kw in (dict(h_fixed=37.0), dict()):
        r = oracle.integrate(m, S, L, w, 0.05, 1e-10, terms=oracle.TERM_ALL & ~oracle.TERM_RR,
                             t_end=5.0e4, phase=True, nthreads=NT, **kw)
        assert (r["status"] == 0).all()
        np.testing.assert_array_equal(r["y"][0], w)
        np.testing.assert_allclose(r["phase"], w * r["t"], rtol=1e-13)


@pytest.mark.parametrize("q,c1,c2", [(1.0, 1.0, 1.0), (3.0, 0.7, -0.4), (8.0, -0.9, 0.2)])
def test_aligned_spins_phase_by_quadrature(q, c1, c2):
    """Spins along L_hat do not precess, so omega-dot depends on omega only
    and Phi* is the integral of omega / omega-dot from omega0 to omega_f."""
    m1, m2 = q / (1 + q), 1 / (1 + q)
    Lh = np.array([0.0, 0.0, 1.0])
    S1, S2 = c1 * m1 ** 2 * Lh, c2 * m2 ** 2 * Lh
    w0, wf = 0.004, 0.05
    m, S, L, w = _one(m1, m2, S1, S2, Lh, w0)
    r = oracle.integrate(m, S, L, w, wf, 1e-12, phase=True)
    assert r["status"][0] == 0

    def w_over_wdot(om):
        y = np.concatenate([[om], S1, S2, Lh]).reshape(10, 1)
        return om / oracle.rhs(m, y)[0, 0]

    exact, _ = si.quad(w_over_wdot, w0, wf, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(r["phase"][0] / exact - 1) < 1e-9


def test_phase_fixed_step_convergence_order_five():
    """Over a stretch where omega grows by ~30 % (so that the phase error is
    well above rounding), halving h divides the phase error by ~2^5."""
    m, S, L, w = _random_pop(8, 15, w0=0.02)
    runs = {}
    hs = (100.0, 50.0, 25.0, 12.5, 0.78125)
    for h in hs:
        r = oracle.integrate(m, S, L, w, 0.2, 1.0, h_fixed=h, t_end=1500.0, phase=True, nthreads=NT)
        assert (r["status"] == 0).all()
        runs[h] = r["phase"]
    err = [np.abs(runs[h] - runs[hs[-1]]).max() for h in hs[:-1]]
    ratios = [err[k] / err[k + 1] for k in range(3)]
    assert all(24 < x < 38 for x in ratios), ratios
    assert ratios[2] > ratios[0]            # approaching 32 from below


def test_phase_leaves_the_step_sequence_unchanged():
    m, S, L, w = _random_pop(64, 21)
    for kw in (dict(), dict(h_fixed=60.0), dict(t_end=2.0e4)):
        a = oracle.integrate(m, S, L, w, 0.05, 1e-9, nthreads=NT, **kw)
        b = oracle.integrate(m, S, L, w, 0.05, 1e-9, phase=True, nthreads=NT, **kw)
        for k in ("y", "t", "steps", "status"):
            np.testing.assert_array_equal(a[k], b[k])
        assert np.isfinite(b["phase"]).all() and (b["phase"] > 0).all()


def test_phase_symmetries():
    """Phi is a scalar: unchanged by exchanging the labels 1 <-> 2 (to the
    tolerance), by a rotation of all vectors, and by the scaling m -> 2m,
    S -> 4S, omega -> omega/2, h -> 2h (dimensionless; exact in binary)."""
    m, S, L, w = _random_pop(16, 16)
    a = oracle.integrate(m, S, L, w, 0.05, 1e-11, phase=True, nthreads=NT)
    b = oracle.integrate(m[::-1].copy(), np.concatenate([S[3:], S[:3]]), L, w, 0.05, 1e-11, phase=True,
                         nthreads=NT)
    np.testing.assert_allclose(a["phase"], b["phase"], rtol=1e-9)
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    c = oracle.integrate(m, S, L, w, 0.05, 1.0, h_fixed=40.0, phase=True, nthreads=NT)
    d = oracle.integrate(m, np.concatenate([Q @ S[:3], Q @ S[3:]]), Q @ L, w, 0.05, 1.0, h_fixed=40.0,
                         phase=True, nthreads=NT)
    np.testing.assert_allclose(c["phase"], d["phase"], rtol=1e-12)
    e = oracle.integrate(2 * m, 4 * S, L, w / 2, 0.025, 1.0, h_fixed=80.0, phase=True, nthreads=NT)
    np.testing.assert_array_equal(e["phase"], c["phase"])


def test_phase_of_done_at_start_and_bad_input_is_zero():
    m, S, L, w = _random_pop(4, 5)
    w[0] = 0.06                  # past omega_f: DONE_AT_START
    m[0, 1] = -1.0               # BAD_INPUT
    r = oracle.integrate(m, S, L, w, 0.05, 1e-9, phase=True)
    assert r["status"][0] == 1 and r["status"][1] == -4
    assert r["phase"][0] == 0.0 and r["phase"][1] == 0.0
    assert (r["phase"][2:] > 0).all()
