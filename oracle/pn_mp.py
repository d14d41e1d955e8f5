"""High-precision (mpmath) evaluation of Eqs. (1)-(4) at single states.

TEST INFRASTRUCTURE.  A second, independent transcription of the right-hand
side with exact rational coefficients, evaluated at 40 significant digits.
It measures the rounding error of the FP64 oracle's right-hand side; it is
not a pin of the transcription by itself (the closed forms, textbook limits
and conservation laws in the tests are).  Readings R1 (theta_hat times eta,
or the literal extra eta), R4 and R5 as in pn_oracle.cpp.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import mpmath as mp

mp.mp.dps = 40


def _q(fr: Fr):
    return mp.mpf(fr.numerator) / fr.denominator


def rhs(m1, m2, y, theta_literal: bool = False):
    """dy/dt at y = (omega, S1[3], S2[3], L[3]); returns a list of 10 mpf."""
    m1, m2 = mp.mpf(m1), mp.mpf(m2)
    y = [mp.mpf(v) for v in y]
    w = y[0]
    S1, S2, L = y[1:4], y[4:7], y[7:10]
    M = m1 + m2
    eta = m1 * m2 / M ** 2
    v = M * w
    pi = mp.pi
    dot = lambda a, b: sum(ai * bi for ai, bi in zip(a, b))
    LS1, LS2, S12 = dot(L, S1), dot(L, S2), dot(S1, S2)
    theta = _q(Fr(1039, 4620))
    third = mp.mpf(1) / 3
    # Eq. (1), with chi_i L.S_hat_i = L.S_i/m_i^2 and chi1 chi2 S_hat.S_hat = S.S/(m1^2 m2^2)
    so = (LS1 / m1 ** 2 * (113 * m1 ** 2 / M ** 2 + 75 * eta)
          + LS2 / m2 ** 2 * (113 * m2 ** 2 / M ** 2 + 75 * eta)) / 12
    ss = eta / 48 * (247 * S12 - 721 * LS1 * LS2) / (m1 ** 2 * m2 ** 2)
    tfac = eta if theta_literal else 1
    c3pn = (_q(Fr(16447322263, 139708800)) - _q(Fr(1712, 105)) * mp.euler + _q(Fr(16, 3)) * pi ** 2
            + (_q(Fr(-273811877, 1088640)) + _q(Fr(451, 48)) * pi ** 2
               - _q(Fr(88, 3)) * theta * tfac) * eta
            + _q(Fr(541, 896)) * eta ** 2 - _q(Fr(5605, 2592)) * eta ** 3
            - _q(Fr(856, 105)) * mp.log(16 * v ** (2 * third)))
    B = (1 - (743 + 924 * eta) / mp.mpf(336) * v ** (2 * third)
         - (so - 4 * pi) * v
         + (_q(Fr(34103, 18144)) + _q(Fr(13661, 2016)) * eta + _q(Fr(59, 18)) * eta ** 2) * v ** (4 * third)
         - ss * v ** (4 * third)
         - (4159 + 15876 * eta) * pi / 672 * v ** (5 * third)
         + c3pn * v ** 2
         + (_q(Fr(-4415, 4032)) + _q(Fr(358675, 6048)) * eta + _q(Fr(91495, 1512)) * eta ** 2) * pi
         * v ** (7 * third))
    wdot = w ** 2 * _q(Fr(96, 5)) * eta * v ** (5 * third) * B
    # Eq. (4) and its 1 <-> 2 image
    pre = v ** 2 / (2 * M)
    Om1 = [pre * (eta * v ** (-third) * (4 + 3 * m2 / m1) * L[c] + (S2[c] - 3 * LS2 * L[c]) / M ** 2)
           for c in range(3)]
    Om2 = [pre * (eta * v ** (-third) * (4 + 3 * m1 / m2) * L[c] + (S1[c] - 3 * LS1 * L[c]) / M ** 2)
           for c in range(3)]
    cross = lambda a, b: [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                          a[0] * b[1] - a[1] * b[0]]
    dS1, dS2 = cross(Om1, S1), cross(Om2, S2)
    dL = [-(v ** third) / (eta * M ** 2) * (dS1[c] + dS2[c]) for c in range(3)]
    return [wdot] + dS1 + dS2 + dL
