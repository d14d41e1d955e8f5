"""The algorithmic FLOP constants of bench.py.

F_RHS and F_STEP_COMB count the arithmetic of Eqs. (1)-(4) and of the
Dormand-Prince tableau with each operation written once (a fused multiply-add
is 2 FLOP, a division 1; special functions not counted); their itemisation
must add up.  The oracle's own counts (its counting scalar: every add, sub,
mul and div of its deliberately plain association, one FLOP each) are
reported beside them and pinned here against the oracle."""
import os
import sys

import numpy as np

import oracle
from paper_0908_3889_amd import population as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_derived_constants_add_up():
    import bench
    assert bench.F_RHS == sum(bench.RHS_FLOP.values()) == 101
    assert bench.F_STEP_COMB == sum(bench.COMB_FLOP.values()) == 586
    # the stage sums: row s of the tableau has s - 1 weights, the 5th-order
    # row (stage 7) has 6 of which b_2 = 0; one FMA per weight and component
    nonzero_a = sum(range(1, 6)) + 5
    assert bench.COMB_FLOP["stage points Y_2..Y_7: 20 nonzero a_sj x 10 components (FMA)"] == nonzero_a * 10 * 2
    assert bench.COMB_FLOP["h a_sj products"] == nonzero_a
    # the error weights b - bhat: e_2 = 0, the other six nonzero (one MUL, five FMA)
    assert bench.COMB_FLOP["error estimate sum_j (b_j - bhat_j) k_j: 10 x (MUL + 5 FMA)"] == 10 * (1 + 5 * 2)
    # common subexpressions only lower the count below the oracle's plain one
    assert bench.F_RHS < bench.ORACLE_F_RHS and bench.F_STEP_COMB < bench.ORACLE_F_STEP_COMB


def test_oracle_constants_match_the_oracle_count():
    import bench
    pop = P.generate("q1to4_1M", 16)
    for i in range(16):
        y0 = np.concatenate([pop["omega0"][i:i + 1], pop["S"][:, i], pop["L"][:, i]])
        c = oracle.count_ops(pop["m"][:, i], y0, pop["omega_f"], pop["tol"])
        r, u = c["rhs"], c["run"]
        assert r["add"] + r["mul"] + r["div"] == bench.ORACLE_F_RHS
        assert (r["cbrt"], r["log"]) == (1, 1)
        attempted = (c["nrhs"] - 1) // 6
        total = u["add"] + u["mul"] + u["div"]
        per_step = (total - c["nrhs"] * bench.ORACLE_F_RHS) / attempted
        # the omega-mode scalings and the few rejected steps move it by < 0.1 %
        assert abs(per_step / bench.ORACLE_F_STEP_COMB - 1) < 1e-3, per_step
        # bench's formula reproduces the oracle's total to the same accuracy
        steps = np.array([[c["accepted"]], [c["rejected"]], [c["nrhs"]]])
        got = bench.algorithmic_flops(steps, bench.ORACLE_F_RHS, bench.ORACLE_F_STEP_COMB)
        assert abs(got / total - 1) < 1e-3
