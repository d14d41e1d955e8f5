"""The algorithmic FLOP constants used by bench.py are the oracle's own
operation counts (state-dependent add/sub/mul/div, one FLOP each)."""
import os
import sys

import numpy as np

import oracle
from paper_0908_3889_amd import population as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_flop_constants_match_the_oracle_count():
    import bench
    pop = P.generate("q1to4_1M", 16)
    for i in range(16):
        y0 = np.concatenate([pop["omega0"][i:i + 1], pop["S"][:, i], pop["L"][:, i]])
        c = oracle.count_ops(pop["m"][:, i], y0, pop["omega_f"], pop["tol"])
        r, u = c["rhs"], c["run"]
        assert r["add"] + r["mul"] + r["div"] == bench.F_RHS
        assert (r["cbrt"], r["log"]) == (1, 1)
        attempted = (c["nrhs"] - 1) // 6
        total = u["add"] + u["mul"] + u["div"]
        per_step = (total - c["nrhs"] * bench.F_RHS) / attempted
        # the omega-mode scalings and the few rejected steps move it by < 0.1 %
        assert abs(per_step / bench.F_STEP_COMB - 1) < 1e-3, per_step
        # bench's formula reproduces the oracle's total to the same accuracy
        steps = np.array([[c["accepted"]], [c["rejected"]], [c["nrhs"]]])
        assert abs(bench.algorithmic_flops(steps) / total - 1) < 1e-3
