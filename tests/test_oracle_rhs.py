"""Pins of the oracle's right-hand side, Eqs. (1)-(4), against things other
than itself: textbook forms of the same physics written in other variables,
exact symmetries, and the rounding level of a 40-digit evaluation.

CPU only.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import pn_mp

HERE = os.path.dirname(os.path.abspath(__file__))


def _state(m1, m2, chi1, chi2, s1, s2, L, w):
    s1 = np.asarray(s1, float) / np.linalg.norm(s1)
    s2 = np.asarray(s2, float) / np.linalg.norm(s2)
    L = np.asarray(L, float) / np.linalg.norm(L)
    return np.concatenate([[w], chi1 * m1 ** 2 * s1, chi2 * m2 ** 2 * s2, L])


def _rhs1(m1, m2, y, **kw):
    return oracle.rhs(np.array([[m1], [m2]]), np.asarray(y).reshape(10, 1), **kw)[:, 0]


def _random_states(rng, n):
    out = []
    for _ in range(n):
        q = rng.uniform(1, 10)
        m1, m2 = q / (1 + q), 1 / (1 + q)
        s1, s2, L = rng.normal(size=(3, 3))
        out.append((m1, m2, _state(m1, m2, rng.uniform(0, 1), rng.uniform(0, 1), s1, s2, L,
                                   rng.uniform(0.002, 0.1))))
    return out


# ---------------------------------------------------------------------------
# Non-spinning omega-dot against the textbook 3.5PN expansion in x=(M w)^{2/3}
# ---------------------------------------------------------------------------

def _taylor_t4_nonspinning(eta, x):
    """dx/dt * M for a circular, non-spinning binary (Blanchet, Living Rev.
    Relativ. 17 (2014) 2, energy-balance expansion): written in x, with the
    3PN eta coefficient as the single rational -56198689/217728 + 451 pi^2/48
    and the log as ln(16 x)."""
    pi, g = mp.pi, mp.euler
    F = lambda a, b: mp.mpf(a) / b
    br = (1 + (F(-743, 336) - F(11, 4) * eta) * x + 4 * pi * x ** F(3, 2)
          + (F(34103, 18144) + F(13661, 2016) * eta + F(59, 18) * eta ** 2) * x ** 2
          + (F(-4159, 672) - F(189, 8) * eta) * pi * x ** F(5, 2)
          + (F(16447322263, 139708800) + F(16, 3) * pi ** 2 - F(1712, 105) * g
             - F(856, 105) * mp.log(16 * x)
             + (F(-56198689, 217728) + F(451, 48) * pi ** 2) * eta
             + F(541, 896) * eta ** 2 - F(5605, 2592) * eta ** 3) * x ** 3
          + (F(-4415, 4032) + F(358675, 6048) * eta + F(91495, 1512) * eta ** 2) * pi * x ** F(7, 2))
    return F(64, 5) * eta * x ** 5 * br


@pytest.mark.parametrize("q", [1.0, 2.5, 4.0, 10.0])
@pytest.mark.parametrize("w", [0.002, 0.01, 0.05, 0.1])
def test_nonspinning_omegadot_matches_textbook_expansion(q, w):
    mp.mp.dps = 30
    m1, m2 = q / (1 + q), 1 / (1 + q)
    M = m1 + m2
    eta = mp.mpf(m1) * m2 / M ** 2
    x = (mp.mpf(M) * w) ** (mp.mpf(2) / 3)
    # omega = x^{3/2}/M  =>  d omega/dt = (3/2) x^{1/2} (dx/dt) / M
    ref = mp.mpf(3) / 2 * mp.sqrt(x) * _taylor_t4_nonspinning(eta, x) / M ** 2
    y = np.array([w] + [0.0] * 6 + [0.0, 0.0, 1.0])
    got = _rhs1(m1, m2, y)[0]
    assert abs(got / float(ref) - 1) < 2e-14


# ---------------------------------------------------------------------------
# Aligned spins: the 1.5PN spin-orbit coefficient in the (chi_s, chi_a, delta)
# form used for aligned-spin templates, and the 2PN spin-spin value.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q,chi1,chi2", [(1.0, 0.9, 0.3), (3.0, 0.5, -0.8), (7.0, -1.0, 1.0)])
def test_aligned_spin_orbit_coefficient(q, chi1, chi2):
    """With S_i along +-L, omega-dot's 1.5PN term is (4 pi - beta) x^{3/2}
    with beta = 113/12 (chi_s + delta chi_a) - 19/3 eta chi_s, delta =
    (m1-m2)/M, chi_s,a = (chi1 +- chi2)/2 (signed chi along L)."""
    m1, m2 = q / (1 + q), 1 / (1 + q)
    eta = m1 * m2
    delta = m1 - m2
    chis, chia = (chi1 + chi2) / 2, (chi1 - chi2) / 2
    beta = 113.0 / 12 * (chis + delta * chia) - 19.0 / 3 * eta * chis
    w = 0.03
    x3 = w  # (M w)^{3/3} with M = 1
    L = np.array([0.0, 0.0, 1.0])
    y = np.concatenate([[w], chi1 * m1 ** 2 * L, chi2 * m2 ** 2 * L, L])
    y0 = np.concatenate([[w], np.zeros(6), L])
    terms = oracle.TERM_RR | oracle.TERM_SO_WDOT | oracle.TERM_PN
    d_spin = _rhs1(m1, m2, y, terms=terms)[0]
    d_none = _rhs1(m1, m2, y0, terms=terms)[0]
    pref = w ** 2 * 96 / 5 * eta * w ** (5 / 3)
    assert abs((d_spin - d_none) / pref - (-beta * x3)) < 1e-13


@pytest.mark.parametrize("geom", ["aligned", "anti", "perp"])
def test_spin_spin_angle_structure(geom):
    """2PN spin-spin term: -(eta/48) chi1 chi2 (247 S1h.S2h - 721 (L.S1h)(L.S2h)) (M w)^{4/3}.
    Three geometries separate the two angular structures."""
    m1, m2, chi1, chi2, w = 0.7, 0.3, 0.8, 0.6, 0.04
    L = np.array([0.0, 0.0, 1.0])
    if geom == "aligned":
        s1, s2 = L, L
    elif geom == "anti":
        s1, s2 = L, -L
    else:
        s1, s2 = np.array([1.0, 0, 0]), np.array([1.0, 0, 0])
    # anti: S1h.S2h = -1, (L.S1h)(L.S2h) = -1  ->  -247 + 721
    expected_bracket = {"aligned": 247 - 721, "anti": -247 + 721, "perp": 247}[geom]
    y = np.concatenate([[w], chi1 * m1 ** 2 * s1, chi2 * m2 ** 2 * s2, L])
    y0 = np.concatenate([[w], np.zeros(6), L])
    terms = oracle.TERM_RR | oracle.TERM_SS_WDOT
    eta = m1 * m2
    pref = w ** 2 * 96 / 5 * eta * w ** (5 / 3)
    diff = (_rhs1(m1, m2, y, terms=terms)[0] - _rhs1(m1, m2, y0, terms=terms)[0]) / pref
    assert abs(diff - (-eta / 48 * chi1 * chi2 * expected_bracket * w ** (4 / 3))) < 1e-14


# ---------------------------------------------------------------------------
# Precession against the textbook form in orbital separation r
# ---------------------------------------------------------------------------

def test_precession_matches_separation_form():
    """Omega_1 = (1/r^3) [ (2 + 3 m2/(2 m1)) L_N + S2/2 - (3/2)(S2.L_hat) L_hat ],
    L_N = mu sqrt(M r) L_hat, r = M (M w)^{-2/3}; dL_hat/dt = -(dS1+dS2)/|L_N|
    (Kidder 1995, leading spin-orbit and spin-spin precession)."""
    rng = np.random.default_rng(5)
    for m1, m2, y in _random_states(rng, 20):
        M = m1 + m2
        w = y[0]
        S1, S2, L = y[1:4], y[4:7], y[7:10]
        r = M * (M * w) ** (-2.0 / 3.0)
        LN = m1 * m2 / M * np.sqrt(M * r)
        Om1 = ((2 + 1.5 * m2 / m1) * LN * L + 0.5 * S2 - 1.5 * np.dot(S2, L) * L) / r ** 3
        Om2 = ((2 + 1.5 * m1 / m2) * LN * L + 0.5 * S1 - 1.5 * np.dot(S1, L) * L) / r ** 3
        dS1, dS2 = np.cross(Om1, S1), np.cross(Om2, S2)
        dL = -(dS1 + dS2) / LN
        got = _rhs1(m1, m2, y)
        scale = np.abs(np.concatenate([dS1, dS2])).max()
        assert np.abs(got[1:4] - dS1).max() < 1e-13 * scale
        assert np.abs(got[4:7] - dS2).max() < 1e-13 * scale
        assert np.abs(got[7:10] - dL).max() < 1e-13 * np.abs(dL).max()


# ---------------------------------------------------------------------------
# Symmetries of Eqs. (1)-(4)
# ---------------------------------------------------------------------------

def test_label_swap_symmetry():
    rng = np.random.default_rng(1)
    for m1, m2, y in _random_states(rng, 20):
        ys = np.concatenate([y[:1], y[4:7], y[1:4], y[7:]])
        a, b = _rhs1(m1, m2, y), _rhs1(m2, m1, ys)
        assert abs(a[0] / b[0] - 1) < 1e-14
        np.testing.assert_allclose(a[1:4], b[4:7], rtol=1e-12, atol=1e-22)
        np.testing.assert_allclose(a[4:7], b[1:4], rtol=1e-12, atol=1e-22)
        np.testing.assert_allclose(a[7:], b[7:], rtol=1e-12, atol=1e-22)


def test_rotation_covariance():
    rng = np.random.default_rng(2)
    for m1, m2, y in _random_states(rng, 20):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        yr = np.concatenate([y[:1], Q @ y[1:4], Q @ y[4:7], Q @ y[7:]])
        a, b = _rhs1(m1, m2, y), _rhs1(m1, m2, yr)
        assert abs(a[0] / b[0] - 1) < 1e-13
        for s in (slice(1, 4), slice(4, 7), slice(7, 10)):
            np.testing.assert_allclose(Q @ a[s], b[s], rtol=0, atol=1e-13 * np.abs(a[s]).max())


def test_scale_invariance():
    """M -> lam M, S -> lam^2 S, omega -> omega/lam (Sec. II: the problem is
    scale free): omega-dot -> omega-dot/lam^2, dS/dt -> lam dS/dt,
    dL/dt -> dL/dt / lam.  lam = 2 scales every rounding exactly."""
    rng = np.random.default_rng(3)
    for lam in (2.0, 0.5):
        for m1, m2, y in _random_states(rng, 10):
            ys = np.concatenate([y[:1] / lam, lam ** 2 * y[1:7], y[7:]])
            a, b = _rhs1(m1, m2, y), _rhs1(lam * m1, lam * m2, ys)
            assert b[0] == a[0] / lam ** 2
            np.testing.assert_array_equal(b[1:7], lam * a[1:7])
            np.testing.assert_array_equal(b[7:], a[7:] / lam)


def test_lhat_dot_perpendicular_and_spin_norms_fixed():
    """L_hat . dL_hat/dt = 0 and S_i . dS_i/dt = 0 identically."""
    rng = np.random.default_rng(4)
    for m1, m2, y in _random_states(rng, 20):
        d = _rhs1(m1, m2, y)
        assert abs(np.dot(y[7:], d[7:])) < 1e-15 * np.linalg.norm(d[7:])
        assert abs(np.dot(y[1:4], d[1:4])) < 1e-15 * np.linalg.norm(d[1:4]) * np.linalg.norm(y[1:4])
        assert abs(np.dot(y[4:7], d[4:7])) < 1e-15 * np.linalg.norm(d[4:7]) * np.linalg.norm(y[4:7])


def test_theta_hat_reading_difference():
    """Reading R1 vs the literal print differ by (88/3) theta_hat (eta - eta^2) x^6
    inside the bracket."""
    m1, m2, w = 0.5, 0.5, 0.05
    y = np.array([w] + [0.0] * 6 + [0.0, 0.0, 1.0])
    a = _rhs1(m1, m2, y)[0]
    b = _rhs1(m1, m2, y, theta_literal=1)[0]
    eta = 0.25
    pref = w ** 2 * 96 / 5 * eta * w ** (5 / 3)
    assert abs((b - a) / pref - 88 / 3 * 1039 / 4620 * (eta - eta ** 2) * w ** 2) < 1e-14


# ---------------------------------------------------------------------------
# Rounding level against the 40-digit evaluation
# ---------------------------------------------------------------------------

def test_rhs_rounding_against_40_digit_points():
    with open(os.path.join(HERE, "golden", "rhs_points.json")) as f:
        pts = json.load(f)["points"]
    for p in pts:
        got = _rhs1(p["m"][0], p["m"][1], np.array(p["y"]), theta_literal=p["theta_literal"])
        ref = np.array([float(v) for v in p["dydt"]])
        assert abs(got[0] / ref[0] - 1) < 1e-14
        for s in (slice(1, 4), slice(4, 7), slice(7, 10)):
            assert np.abs(got[s] - ref[s]).max() <= 1e-14 * np.abs(ref[s]).max() + 1e-300


def test_rhs_rounding_random_states():
    rng = np.random.default_rng(6)
    for m1, m2, y in _random_states(rng, 10):
        got = _rhs1(m1, m2, y)
        ref = np.array([float(v) for v in pn_mp.rhs(m1, m2, list(y))])
        assert abs(got[0] / ref[0] - 1) < 1e-14
        for s in (slice(1, 4), slice(4, 7), slice(7, 10)):
            assert np.abs(got[s] - ref[s]).max() <= 1e-14 * np.abs(ref[s]).max()
