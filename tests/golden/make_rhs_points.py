"""Write rhs_points.json: Eqs. (1)-(4) at a few states, to 40 digits.

Calls only the oracle's high-precision transcription (oracle/pn_mp.py).
Run from the repository root:  python tests/golden/make_rhs_points.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mpmath as mp  # noqa: E402

from oracle import pn_mp  # noqa: E402

mp.mp.dps = 40


def state(m1, m2, chi1, chi2, s1, s2, L, w):
    S1 = [chi1 * m1 ** 2 * c for c in s1]
    S2 = [chi2 * m2 ** 2 * c for c in s2]
    return [w] + S1 + S2 + list(L)


POINTS = [
    # m1, m2, state, theta_literal
    (0.6, 0.4, state(0.6, 0.4, 0.9, 0.5, (0.6, 0.0, 0.8), (0.0, -0.8, 0.6), (0.0, 0.6, 0.8), 0.02), 0),
    (0.6, 0.4, state(0.6, 0.4, 0.9, 0.5, (0.6, 0.0, 0.8), (0.0, -0.8, 0.6), (0.0, 0.6, 0.8), 0.02), 1),
    (0.5, 0.5, state(0.5, 0.5, 1.0, 1.0, (0.48, 0.64, 0.6), (-0.36, 0.0, 0.8), (0.0, 0.0, 1.0), 0.004), 0),
    (0.8, 0.2, state(0.8, 0.2, 0.3, 0.95, (0.0, 0.0, -1.0), (0.28, -0.96, 0.0), (0.6, 0.0, 0.8), 0.049), 0),
    (10.0 / 11.0, 1.0 / 11.0, state(10.0 / 11.0, 1.0 / 11.0, 0.7, 0.1, (0.8, 0.6, 0.0),
                                      (0.0, 0.6, -0.8), (0.0, 0.0, 1.0), 0.002), 0),
]


def main():
    out = []
    for m1, m2, y, lit in POINTS:
        d = pn_mp.rhs(m1, m2, y, theta_literal=bool(lit))
        out.append({"m": [m1, m2], "y": y, "theta_literal": lit,
                    "dydt": [mp.nstr(v, 40) for v in d]})
    with open(os.path.join(HERE, "rhs_points.json"), "w") as f:
        json.dump({"source": "Eqs. (1)-(4) evaluated at 40 digits by oracle/pn_mp.py",
                   "points": out}, f, indent=1)


if __name__ == "__main__":
    main()
