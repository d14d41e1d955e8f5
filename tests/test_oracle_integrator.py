"""Pins of the oracle's integrator (Dormand-Prince from omega0 to omega_f,
Sec. II) against closed forms, conservation laws, convergence order, an
independent library integrator and the paper's printed statistics (Sec. V).

CPU only.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy import integrate as si

import oracle
from paper_0908_3889_amd import population as P

NT = 8


def _pop(m1, m2, S1, S2, L, w0):
    n = len(m1)
    return (np.stack([m1, m2]), np.concatenate([S1, S2]).reshape(6, n), np.asarray(L).reshape(3, n),
            np.asarray(w0, float))


def _one(m1, m2, S1, S2, L, w0):
    return (np.array([[m1], [m2]]), np.concatenate([S1, S2]).reshape(6, 1),
            np.asarray(L, float).reshape(3, 1), np.array([w0]))


# ---------------------------------------------------------------------------
# Tableau: exact order conditions
# ---------------------------------------------------------------------------

def _fr(pair):
    return Fr(int(pair[0]), int(pair[1]))


def test_dormand_prince_order_conditions():
    a, b, bh, c = oracle.tableau()
    A = [[_fr(a[i, j]) for j in range(6)] + [Fr(0)] for i in range(7)]
    B = [_fr(x) for x in b]
    BH = [_fr(x) for x in bh]
    Cc = [_fr(x) for x in c]
    s = range(7)
    for i in s:
        assert sum(A[i][:i]) == Cc[i]                       # row sums
    assert [A[6][j] for j in range(6)] == B[:6] and B[6] == 0   # FSAL

    def conds(w):
        Ac = [sum(A[i][j] * Cc[j] for j in s) for i in s]
        Ac2 = [sum(A[i][j] * Cc[j] ** 2 for j in s) for i in s]
        AAc = [sum(A[i][j] * Ac[j] for j in s) for i in s]
        Ac3 = [sum(A[i][j] * Cc[j] ** 3 for j in s) for i in s]
        AcAc = [sum(A[i][j] * Cc[j] * Ac[j] for j in s) for i in s]
        AAc2 = [sum(A[i][j] * Ac2[j] for j in s) for i in s]
        AAAc = [sum(A[i][j] * AAc[j] for j in s) for i in s]
        S = lambda f: sum(w[i] * f(i) for i in s)
        o = {}
        o[1] = [S(lambda i: 1) - 1]
        o[2] = [S(lambda i: Cc[i]) - Fr(1, 2)]
        o[3] = [S(lambda i: Cc[i] ** 2) - Fr(1, 3), S(lambda i: Ac[i]) - Fr(1, 6)]
        o[4] = [S(lambda i: Cc[i] ** 3) - Fr(1, 4), S(lambda i: Cc[i] * Ac[i]) - Fr(1, 8),
                S(lambda i: Ac2[i]) - Fr(1, 12), S(lambda i: AAc[i]) - Fr(1, 24)]
        o[5] = [S(lambda i: Cc[i] ** 4) - Fr(1, 5), S(lambda i: Cc[i] ** 2 * Ac[i]) - Fr(1, 10),
                S(lambda i: Cc[i] * Ac2[i]) - Fr(1, 15), S(lambda i: Cc[i] * AAc[i]) - Fr(1, 30),
                S(lambda i: Ac[i] ** 2) - Fr(1, 20), S(lambda i: Ac3[i]) - Fr(1, 20),
                S(lambda i: AcAc[i]) - Fr(1, 40), S(lambda i: AAc2[i]) - Fr(1, 60),
                S(lambda i: AAAc[i]) - Fr(1, 120)]
        return o

    ob = conds(B)
    assert sum(len(v) for v in ob.values()) == 17
    assert all(x == 0 for v in ob.values() for x in v)
    oh = conds(BH)
    assert all(x == 0 for k in (1, 2, 3, 4) for x in oh[k])
    assert any(x != 0 for x in oh[5])


# ---------------------------------------------------------------------------
# Closed form: leading-order (Newtonian) chirp
# ---------------------------------------------------------------------------

def _newtonian(q, w0):
    m1, m2 = q / (1 + q), 1 / (1 + q)
    z = np.zeros(3)
    return _one(m1, m2, z, z, [0, 0, 1.0], w0), m1 * m2


@pytest.mark.parametrize("q,w0,wf", [(1.0, 0.01, 0.05), (1.0, 0.005, 0.05), (4.0, 0.005, 0.05),
                                     (10.0, 0.002, 0.05)])
def test_newtonian_chirp_time_to_omega_f(q, w0, wf):
    """omega(t) = [w0^{-8/3} - (256/5) eta M^{5/3} t]^{-3/8}, so
    t* = (w0^{-8/3} - wf^{-8/3}) / ((256/5) eta M^{5/3})."""
    (m, S, L, w), eta = _newtonian(q, w0)
    t_star = (w0 ** (-8 / 3) - wf ** (-8 / 3)) / (256 / 5 * eta)
    errs = []
    for tol in (1e-10, 1e-11, 1e-12, 1e-13):
        r = oracle.integrate(m, S, L, w, wf, tol, terms=oracle.TERM_RR)
        assert r["status"][0] == 0
        assert r["y"][0, 0] == wf
        errs.append(abs(r["t"][0] / t_star - 1))
    # converges to the closed form as the tolerance shrinks
    assert errs[-1] < 1e-10
    assert all(errs[k + 1] < errs[k] / 5 for k in range(3)), errs


@pytest.mark.parametrize("frac", [0.3, 0.9, 0.999])
def test_newtonian_chirp_omega_at_time(frac):
    q, w0, wf = 2.0, 0.004, 0.1
    (m, S, L, w), eta = _newtonian(q, w0)
    tc = w0 ** (-8 / 3) / (256 / 5 * eta)            # coalescence time
    t_end = frac * tc
    exact = (w0 ** (-8 / 3) - 256 / 5 * eta * t_end) ** (-3 / 8)
    errs = []
    for tol in (1e-11, 1e-12, 1e-13):
        r = oracle.integrate(m, S, L, w, wf, tol, terms=oracle.TERM_RR, t_end=t_end)
        assert r["status"][0] == 0
        assert r["t"][0] == pytest.approx(t_end, rel=1e-15)
        errs.append(abs(r["y"][0, 0] / exact - 1))
    assert errs[-1] < 5e-9
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10, errs


# ---------------------------------------------------------------------------
# Aligned spins: a fixed point of the precession; t* by quadrature
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q,c1,c2", [(1.0, 1.0, 1.0), (3.0, 0.7, -0.4), (8.0, -0.9, 0.2)])
def test_aligned_spins_time_by_quadrature(q, c1, c2):
    m1, m2 = q / (1 + q), 1 / (1 + q)
    Lh = np.array([0.0, 0.0, 1.0])
    S1, S2 = c1 * m1 ** 2 * Lh, c2 * m2 ** 2 * Lh
    w0, wf = 0.004, 0.05
    m, S, L, w = _one(m1, m2, S1, S2, Lh, w0)
    r = oracle.integrate(m, S, L, w, wf, 1e-12)
    assert r["status"][0] == 0
    np.testing.assert_array_equal(r["y"][1:, 0], np.concatenate([S1, S2, Lh]))

    def inv_wdot(om):
        y = np.concatenate([[om], S1, S2, Lh]).reshape(10, 1)
        return 1.0 / oracle.rhs(m, y)[0, 0]

    t_star, _ = si.quad(inv_wdot, w0, wf, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(r["t"][0] / t_star - 1) < 1e-9


# ---------------------------------------------------------------------------
# Conservation laws
# ---------------------------------------------------------------------------

def _random_pop(n, seed, q=(1, 4), chi=(0.3, 1.0), w0=0.005):
    rng = np.random.default_rng(seed)
    qq = rng.uniform(*q, n)
    m1, m2 = qq / (1 + qq), 1 / (1 + qq)
    u = rng.normal(size=(3, 3, n))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    c1, c2 = rng.uniform(*chi, n), rng.uniform(*chi, n)
    S1, S2, L = c1 * m1 ** 2 * u[0], c2 * m2 ** 2 * u[1], u[2]
    return np.stack([m1, m2]), np.concatenate([S1, S2]), L, np.full(n, w0)


def test_spin_and_lhat_norms_conserved():
    """|S1|, |S2| and |L_hat| are constants of Eqs. (2)-(3); the drift stays
    within the local tolerance summed over the steps, and shrinks with it."""
    m, S, L, w = _random_pop(32, 11)
    drift = []
    for tol in (1e-9, 1e-11):
        r = oracle.integrate(m, S, L, w, 0.05, tol, nthreads=NT)
        assert (r["status"] == 0).all()
        y = r["y"]
        d = np.stack([np.abs(np.linalg.norm(y[1:4], axis=0) - np.linalg.norm(S[:3], axis=0)),
                      np.abs(np.linalg.norm(y[4:7], axis=0) - np.linalg.norm(S[3:], axis=0)),
                      np.abs(np.linalg.norm(y[7:], axis=0) - 1)])
        assert (d <= tol * r["steps"][0]).all()
        drift.append(d.max())
    assert drift[1] < drift[0] / 20


def test_total_angular_momentum_conserved_without_radiation_reaction():
    """J = eta M^{5/3} omega^{-1/3} L_hat + S1 + S2, |L_N| as given after Eq. (3);
    with omega-dot switched off, dJ/dt = 0."""
    m, S, L, w = _random_pop(16, 12, w0=0.02)
    terms = oracle.TERM_ALL & ~oracle.TERM_RR
    r = oracle.integrate(m, S, L, w, 0.05, 1e-11, terms=terms, t_end=3000.0, nthreads=NT)
    assert (r["status"] == 0).all()
    eta = m[0] * m[1]
    J0 = eta * w ** (-1 / 3) * L + S[:3] + S[3:]
    y = r["y"]
    J1 = eta * y[0] ** (-1 / 3) * y[7:] + y[1:4] + y[4:7]
    assert np.abs(J1 - J0).max() < 1e-9 * np.abs(J0).max()
    # the motion is not trivial: L_hat moved
    assert np.abs(y[7:] - L).max() > 1e-2


def test_projected_spin_conserved_without_spin_spin_precession():
    """With only the L_hat part of Eq. (4), (4 + 3 m2/m1) L.S1 + (4 + 3 m1/m2) L.S2
    is conserved, with radiation reaction on."""
    m, S, L, w = _random_pop(16, 13)
    terms = oracle.TERM_ALL & ~oracle.TERM_SS_PREC
    r = oracle.integrate(m, S, L, w, 0.05, 1e-11, terms=terms, nthreads=NT)
    assert (r["status"] == 0).all()
    m1, m2 = m
    f = lambda S1, S2, Lh: ((4 + 3 * m2 / m1) * (Lh * S1).sum(0) + (4 + 3 * m1 / m2) * (Lh * S2).sum(0))
    y = r["y"]
    c0, c1 = f(S[:3], S[3:], L), f(y[1:4], y[4:7], y[7:])
    assert np.abs(c1 - c0).max() < 1e-9
    # with the spin-spin part on, it is not conserved
    r2 = oracle.integrate(m, S, L, w, 0.05, 1e-11, nthreads=NT)
    y2 = r2["y"]
    assert np.abs(f(y2[1:4], y2[4:7], y2[7:]) - c0).max() > 1e-4


def test_equal_mass_spin_dot_conserved_without_spin_spin_precession():
    """m1 = m2 and no spin-spin precession: S1.S2 is conserved (the reason for
    the high initial-final correlation of S1_hat.S2_hat, Sec. V A)."""
    m, S, L, w = _random_pop(16, 14, q=(1, 1))
    terms = oracle.TERM_ALL & ~oracle.TERM_SS_PREC
    r = oracle.integrate(m, S, L, w, 0.05, 1e-11, terms=terms, nthreads=NT)
    y = r["y"]
    d0 = (S[:3] * S[3:]).sum(0)
    d1 = (y[1:4] * y[4:7]).sum(0)
    assert np.abs(d1 - d0).max() < 1e-10


# ---------------------------------------------------------------------------
# Convergence order 5 of the fixed-step scheme
# ---------------------------------------------------------------------------

def test_fixed_step_convergence_order_five():
    m, S, L, w = _random_pop(8, 15, w0=0.01)
    t_end = 4000.0
    runs = {}
    for h in (200.0, 100.0, 50.0, 25.0, 1.5625):
        r = oracle.integrate(m, S, L, w, 0.05, 1.0, h_fixed=h, t_end=t_end, nthreads=NT)
        assert (r["status"] == 0).all()
        runs[h] = r["y"]
    ref = runs[1.5625]
    err = [np.abs(runs[h] - ref).max() for h in (200.0, 100.0, 50.0, 25.0)]
    ratios = [err[k] / err[k + 1] for k in range(3)]
    # global error O(h^5): halving h divides it by 2^5 = 32
    assert all(27 < x < 38 for x in ratios), ratios


# ---------------------------------------------------------------------------
# Symmetries of the integration
# ---------------------------------------------------------------------------

def test_label_swap_of_whole_integration():
    m, S, L, w = _random_pop(16, 16)
    a = oracle.integrate(m, S, L, w, 0.05, 1e-10, nthreads=NT)
    b = oracle.integrate(m[::-1].copy(), np.concatenate([S[3:], S[:3]]), L, w, 0.05, 1e-10,
                         nthreads=NT)
    ya, yb = a["y"], b["y"]
    np.testing.assert_allclose(ya[1:4], yb[4:7], atol=1e-10)
    np.testing.assert_allclose(ya[4:7], yb[1:4], atol=1e-10)
    np.testing.assert_allclose(ya[7:], yb[7:], atol=1e-10)
    np.testing.assert_allclose(a["t"], b["t"], rtol=1e-11)


def test_rotation_of_whole_integration_fixed_step():
    m, S, L, w = _random_pop(8, 17)
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    a = oracle.integrate(m, S, L, w, 0.05, 1.0, h_fixed=40.0, nthreads=NT)
    b = oracle.integrate(m, np.concatenate([Q @ S[:3], Q @ S[3:]]), Q @ L, w, 0.05, 1.0,
                         h_fixed=40.0, nthreads=NT)
    for s in (slice(1, 4), slice(4, 7), slice(7, 10)):
        np.testing.assert_allclose(Q @ a["y"][s], b["y"][s], atol=1e-11)
    da, db = oracle.observables(a["y"]), oracle.observables(b["y"])
    np.testing.assert_allclose(da, db, atol=1e-11)


def test_scale_invariance_of_whole_integration():
    """m -> 2m, S -> 4S, omega -> omega/2, h -> 2h gives t -> 2t and identical
    unit-vector dot products, to the last bit (Sec. II: scale free)."""
    m, S, L, w = _random_pop(8, 18)
    a = oracle.integrate(m, S, L, w, 0.05, 1.0, h_fixed=40.0, nthreads=NT)
    b = oracle.integrate(2 * m, 4 * S, L, w / 2, 0.025, 1.0, h_fixed=80.0, nthreads=NT)
    np.testing.assert_array_equal(b["t"], 2 * a["t"])
    np.testing.assert_array_equal(b["y"][1:7], 4 * a["y"][1:7])
    np.testing.assert_array_equal(b["y"][7:], a["y"][7:])


# ---------------------------------------------------------------------------
# Independent library integrator with a terminal event at omega_f
# ---------------------------------------------------------------------------

def test_against_scipy_dop853_with_terminal_event():
    """SciPy's DOP853 (an 8th-order Dormand-Prince pair) with a terminal event
    at omega = omega_f gives the final state independently of this
    integrator's stepper, controller and omega-step termination.  The
    oracle's final dot products converge to it as tol shrinks (about
    linearly in tol) and agree to 2e-9 at tol = 1e-14."""
    m, S, L, w = _random_pop(8, 19, q=(1, 4), chi=(0, 1), w0=0.005)
    tols = (1e-10, 1e-11, 1e-12, 1e-13, 1e-14)
    runs = [oracle.integrate(m, S, L, w, 0.05, tol, nthreads=NT) for tol in tols]
    dots = [oracle.observables(r["y"]) for r in runs]
    for i in range(m.shape[1]):
        mm = m[:, i:i + 1]

        def f(t, y):
            return oracle.rhs(mm, y.reshape(10, 1))[:, 0]

        ev = lambda t, y: y[0] - 0.05
        ev.terminal, ev.direction = True, 1
        y0 = np.concatenate([[w[i]], S[:, i], L[:, i]])
        sol = si.solve_ivp(f, (0, 1e7), y0, method="DOP853", rtol=3e-14, atol=3e-14, events=ev)
        d = oracle.observables(sol.y_events[0][0].reshape(10, 1))[:, 0]
        tf = sol.t_events[0][0]
        errs = [np.abs(d - dd[:, i]).max() for dd in dots]
        assert errs[-1] < 2e-9, errs
        assert all(errs[k + 1] < errs[k] / 5 for k in range(2)), errs
        assert abs(tf / runs[-1]["t"][i] - 1) < 1e-10


# ---------------------------------------------------------------------------
# Step controller: SciPy's RK45, an independent implementation of the same
# Dormand-Prince pair and the same controller
# ---------------------------------------------------------------------------

def _scipy_rk45_t_stretch(m, y0, tol, omega_f, h0):
    """Accepted step sizes of scipy.integrate.RK45 from y0 (first step h0,
    rtol = atol = tol) up to its first step that passes omega_f, and the
    rejections before that step's acceptance (each attempt costs six
    right-hand-side evaluations)."""
    calls = [0]

    def f(t, y):
        calls[0] += 1
        return oracle.rhs(m, y.reshape(10, 1))[:, 0]

    s = si.RK45(f, 0.0, y0, t_bound=1e12, first_step=h0, rtol=tol, atol=tol)
    hs, rej = [], 0
    while True:
        c0 = calls[0]
        assert s.step() is None and s.status == "running"
        attempts, left = divmod(calls[0] - c0, 6)
        assert left == 0
        rej += attempts - 1
        if s.y[0] > omega_f:
            return np.array(hs), rej
        hs.append(s.h_previous)


@pytest.mark.parametrize("workload,h0", [("q1to4_1M", 10.0), ("equal_mass_maxspin_1k", 10.0),
                                         ("q1to4_1M", 2e4)])
def test_step_controller_matches_scipy_rk45(monkeypatch, workload, h0):
    """SciPy's RK45 is the Dormand-Prince 5(4) pair advancing with the
    5th-order solution, with the root-mean-square error norm over the
    components scaled by atol + rtol max(|y|, |y_new|), safety factor 0.9,
    exponent -1/5, smallest factor 0.2 and no growth right after a
    rejection: readings R7 and R8 of Sec. II's "error tolerance".  Its
    largest growth factor is 10 where R8 reads 5; patched to 5, with the
    initial step h = 10 of Sec. II and rtol = atol = tol, its accepted time
    steps up to the step that passes omega_f must be the oracle's, with the
    same rejections.  A first step of 2e4 is rejected by factors of the
    smallest factor, so that clamp is exercised too.

    The step sizes agree to rounding of the error estimate, which is a
    small difference of stage derivatives (at tol = 1e-10 about 1e-7 of
    them), so a different summation order moves the error norm by up to
    ~1e-7 relative and the next step by a fifth of that: measured at most
    3.2e-8 (median 5e-10) over these workloads.  A wrong exponent (-1/4),
    safety factor (0.95), clamp (10 or 0.1) or norm (a max-norm) moves the
    steps by 0.6 % to 300 % and changes the step counts."""
    import scipy.integrate._ivp.rk as rk
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    pop = P.generate(workload, 8)
    r = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                         h0=h0, record=8192, nthreads=NT)
    assert (r["status"] == 0).all()
    n_t, n_w = r["n_tw"]
    rels = []
    for i in range(pop["n"]):
        y0 = np.concatenate([[pop["omega0"][i]], pop["S"][:, i], pop["L"][:, i]])
        hs, rej = _scipy_rk45_t_stretch(pop["m"][:, i:i + 1], y0, pop["tol"], pop["omega_f"], h0)
        assert hs.size == n_t[i]
        rels.append(np.abs(hs / r["h_record"][i, :n_t[i]] - 1))
        # an omega stretch of one step had no rejection, so all of the
        # oracle's rejections are in the time stretch
        if n_w[i] == 1:
            assert rej == r["steps"][1][i]
        else:
            assert rej <= r["steps"][1][i]
    rel = np.concatenate(rels)
    assert rel.max() < 1e-7 and np.median(rel) < 1e-9, (rel.max(), np.median(rel))
    assert (n_w == 1).sum() >= pop["n"] // 2
    if h0 > 10.0:
        assert r["steps"][1].min() >= 2         # the first step is rejected by the smallest factor


def _rhs_in_omega(m, with_t):
    """dY/domega for Y = (omega, S1, S2, L_hat[, t]): (1, f_1/f_0, ..., f_9/f_0[, 1/f_0])."""
    def f(w, Y):
        d = oracle.rhs(m, Y[:10].reshape(10, 1))[:, 0]
        g = np.concatenate([[1.0], d[1:] / d[0]])
        return np.concatenate([g, [1.0 / d[0]]]) if with_t else g
    return f


@pytest.mark.parametrize("workload", ["q1to4_1M", "equal_mass_maxspin_1k", "batching_4M", "paper_timing"])
def test_omega_stretch_matches_scipy_rk45_in_omega(monkeypatch, workload):
    """The final stretch of reading R10: the time step whose accepted
    candidate passes omega_f is discarded, and the rest is integrated with
    omega as the independent variable, dY/domega = f/f_0, by the same
    Dormand-Prince pair and controller, starting with the whole distance
    left.  On every workload that first omega-step is accepted, so the
    stretch is one step from the state after the recorded time steps to
    omega_f exactly.  SciPy's RK45 started at that state (the recorded time
    steps replayed), with first_step = omega_f - omega and t_bound = omega_f,
    must take the same single step and land on the oracle's final spins and
    L_hat, and, with dt/domega = 1/f_0 carried along, on its t.  A stretch
    integrated in t, a missing 1/f_0, the state of the discarded step or a
    first step other than the distance left all fail it."""
    import scipy.integrate._ivp.rk as rk
    monkeypatch.setattr(rk, "MAX_FACTOR", 5.0)
    pop = P.generate(workload, 8)
    r = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                         record=8192, nthreads=NT)
    assert (r["status"] == 0).all()
    n_t, n_w = r["n_tw"]
    assert (n_w == 1).all()
    assert (r["y"][0] == pop["omega_f"]).all()
    # the state after the recorded time steps (replayed: the adaptive run's arithmetic)
    k = int(n_t.max())
    sw = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                          replay={"h": np.ascontiguousarray(r["h_record"][:, :k]), "n_t": n_t,
                                  "n_w": np.zeros_like(n_w)}, nthreads=NT)
    assert (sw["y"][0] < pop["omega_f"]).all()
    for i in range(pop["n"]):
        m = pop["m"][:, i:i + 1]
        ys, ts, wf = sw["y"][:, i], sw["t"][i], pop["omega_f"]
        s = si.RK45(_rhs_in_omega(m, False), ys[0], ys, t_bound=wf, first_step=wf - ys[0],
                    rtol=pop["tol"], atol=pop["tol"])
        assert s.step() is None and s.status == "finished" and s.t == wf
        assert s.nfev == 7                      # one attempt (FSAL: 1 + 6 evaluations)
        assert np.abs(s.y[1:] - r["y"][1:, i]).max() < 1e-13
        s11 = si.RK45(_rhs_in_omega(m, True), ys[0], np.concatenate([ys, [ts]]), t_bound=wf,
                      first_step=wf - ys[0], rtol=pop["tol"], atol=pop["tol"])
        assert s11.step() is None and s11.status == "finished" and s11.nfev == 7
        assert abs(s11.y[10] / r["t"][i] - 1) < 1e-13


# ---------------------------------------------------------------------------
# Termination and status codes
# ---------------------------------------------------------------------------

def test_termination_lands_exactly_on_omega_f_and_matches_time_mode():
    m, S, L, w = _random_pop(8, 20)
    r = oracle.integrate(m, S, L, w, 0.05, 1e-11, nthreads=NT)
    assert (r["y"][0] == 0.05).all()
    assert (r["n_tw"][1] >= 1).all()           # at least one omega-step each
    for i in range(8):
        s = slice(i, i + 1)
        rt = oracle.integrate(m[:, s], S[:, s], L[:, s], w[s], 0.05, 1e-11, t_end=r["t"][i])
        assert abs(rt["y"][0, 0] - 0.05) < 1e-10
        assert np.abs(rt["y"][1:, 0] - r["y"][1:, i]).max() < 1e-8


def test_status_codes():
    m, S, L, w = _random_pop(6, 21)
    w = w.copy(); m = m.copy(); S = S.copy()
    w[0] = 0.06                     # omega0 >= omega_f
    m[0, 1] = -0.5                  # bad mass
    S[2, 2] = np.nan                # non-finite input
    r = oracle.integrate(m, S, L, w, 0.05, 1e-8, nthreads=1)
    assert r["status"][0] == 1 and (r["steps"][:, 0] == [0, 0, 0]).all()
    np.testing.assert_array_equal(r["y"][:, 0], np.concatenate([[0.06], S[:, 0], L[:, 0]]))
    assert r["status"][1] == -4 and r["status"][2] == -4
    assert (r["status"][3:] == 0).all()
    r = oracle.integrate(m[:, 3:], S[:, 3:], L[:, 3:], w[3:], 0.05, 1e-8, max_steps=3)
    assert (r["status"] == -1).all() and (r["steps"][0] + r["steps"][1] == 3).all()
    r = oracle.integrate(m[:, 3:], S[:, 3:], L[:, 3:], w[3:], 0.05, 1e-300)
    assert (r["status"] == -2).all()
    # overflow inside the right-hand side
    r = oracle.integrate(m[:, 3:4], S[:, 3:4], L[:, 3:4], np.array([1e80]), 0.05, 1e-8,
                         t_end=10.0)
    assert r["status"][0] == -3


def test_record_and_replay_reproduce_the_adaptive_run():
    m, S, L, w = _random_pop(8, 22)
    r = oracle.integrate(m, S, L, w, 0.05, 1e-9, record=4096, nthreads=NT)
    p = oracle.integrate(m, S, L, w, 0.05, 1e-9, replay=r["replay"], nthreads=NT)
    np.testing.assert_array_equal(p["y"], r["y"])
    np.testing.assert_array_equal(p["t"], r["t"])
    np.testing.assert_array_equal(p["steps"][0], r["steps"][0])


def test_tangent_matches_central_differences_in_replay():
    m, S, L, w = _random_pop(4, 23)
    r = oracle.integrate(m, S, L, w, 0.05, 1e-9, record=4096, nthreads=NT)
    rng = np.random.default_rng(0)
    dm, dS, dL = rng.normal(size=(2, 4)), rng.normal(size=(6, 4)) * 0.1, rng.normal(size=(3, 4))
    dw = np.zeros(4)
    tg = oracle.tangent(m, S, L, w, dm, dS, dL, dw, 0.05, 1e-9, r["replay"])
    np.testing.assert_array_equal(tg["y"], r["y"])
    eps = 1e-6
    yp = oracle.integrate(m + eps * dm, S + eps * dS, L + eps * dL, w, 0.05, 1e-9,
                          replay=r["replay"])["y"]
    ym = oracle.integrate(m - eps * dm, S - eps * dS, L - eps * dL, w, 0.05, 1e-9,
                          replay=r["replay"])["y"]
    fd = (yp - ym) / (2 * eps)
    scale = np.abs(tg["dy"]).max(axis=0)
    assert (np.abs(fd - tg["dy"]).max(axis=0) < 1e-6 * scale).all()


# ---------------------------------------------------------------------------
# The paper's printed statistics (Sec. V)
# ---------------------------------------------------------------------------

def _initial_final_r(pop):
    r = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                         nthreads=NT)
    assert (r["status"] == 0).all()
    y0 = np.concatenate([pop["omega0"][None], pop["S"], pop["L"]])
    d0, d1 = oracle.observables(y0), oracle.observables(r["y"])
    return [np.corrcoef(d0[k], d1[k])[0, 1] for k in range(3)], d1


@pytest.mark.slow
def test_paper_equal_mass_maximal_spin_correlations():
    """m_i = 0.5, chi_i = 1, omega 0.00395 -> 0.05: r = 0.99 for S1_hat.S2_hat and
    r = 0.65 for S_i_hat.L_hat (Sec. V A); final S1_hat.S2_hat uniform."""
    pop = P.generate("paper_equal_mass", 4096)
    r, d1 = _initial_final_r(pop)
    assert abs(r[0] - 0.99) < 0.01
    assert abs(r[1] - 0.65) < 0.03 and abs(r[2] - 0.65) < 0.03
    h, _ = np.histogram(d1[0], bins=20, range=(-1, 1))
    chi2 = ((h - 4096 / 20) ** 2 / (4096 / 20)).sum()
    assert chi2 < 45            # 19 dof; p ~ 1e-3


@pytest.mark.slow
def test_paper_equal_spin_correlation_stays_high():
    """Equal masses, chi_1 = chi_2 = chi: r(S1_hat.S2_hat) > 0.98 (Sec. V C)."""
    import dataclasses
    for chi in (0.4, 0.7):
        w = dataclasses.replace(P.WORKLOADS["paper_equal_mass"], chi=("fixed", chi, chi))
        r, _ = _initial_final_r(P.generate(w, 2048))
        assert r[0] > 0.98


@pytest.mark.slow
def test_paper_unequal_mass_low_spin_anticorrelation():
    """m1 = 0.4, chi = 0.05: r = -0.14 (Sec. V D)."""
    import dataclasses
    w = dataclasses.replace(P.WORKLOADS["paper_equal_mass"], q=("fixed", 0.4 / 0.6),
                            chi=("fixed", 0.05, 0.05))
    r, _ = _initial_final_r(P.generate(w, 4096))
    assert abs(r[0] - (-0.14)) < 0.03
