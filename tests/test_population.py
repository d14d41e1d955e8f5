"""The seeded synthetic populations (the inputs of every workload): the
parametrisation of Sec. II (M = 1, m1 = q/(1+q), S_i = chi_i m_i^2 S_hat_i),
isotropic spin directions (Sec. V, Marsaglia), L_hat = z, the stated ranges,
and that a prefix of a population is the same whatever its length."""
import numpy as np
import pytest
from scipy import stats

from paper_0908_3889_amd import population as P


@pytest.mark.parametrize("name", sorted(P.WORKLOADS))
def test_parametrisation_and_ranges(name):
    w = P.WORKLOADS[name]
    n = min(w.n, 65536)
    pop = P.generate(w, n)
    m1, m2 = pop["m"]
    assert pop["m"].shape == (2, n) and pop["S"].shape == (6, n) and pop["L"].shape == (3, n)
    np.testing.assert_allclose(m1 + m2, 1.0, rtol=0, atol=1e-15)
    assert (m1 >= m2).all()
    q = m1 / m2
    if w.q[0] == "uniform":
        assert q.min() >= w.q[1] * (1 - 1e-12) and q.max() <= w.q[2] * (1 + 1e-12)
    else:
        np.testing.assert_allclose(q, w.q[1], rtol=1e-12)
    chi = pop["chi"]
    for i, (mi, s) in enumerate(((m1, pop["S"][:3]), (m2, pop["S"][3:]))):
        np.testing.assert_allclose(np.linalg.norm(s, axis=0), chi[i] * mi ** 2, rtol=1e-14, atol=1e-300)
    if w.chi[0] == "uniform":
        assert chi.min() >= w.chi[1] and chi.max() <= w.chi[2]
    np.testing.assert_array_equal(pop["L"], np.tile([[0.0], [0.0], [1.0]], (1, n)))
    w0 = pop["omega0"]
    if w.omega0[0] == "loguniform":
        assert w0.min() >= w.omega0[1] * (1 - 1e-12) and w0.max() <= w.omega0[2] * (1 + 1e-12)
    assert (w0 < pop["omega_f"]).all() and pop["tol"] == w.tol


def test_spin_directions_are_isotropic():
    """Uniform directions on the sphere: each Cartesian component of S_hat is
    uniform on [-1, 1] (Archimedes), and the two spins are independent."""
    pop = P.generate("q1to4_1M", 200000)
    for s in (pop["S"][:3], pop["S"][3:]):
        u = s / np.linalg.norm(s, axis=0)
        for c in range(3):
            assert stats.kstest(u[c], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    u1 = pop["S"][:3] / np.linalg.norm(pop["S"][:3], axis=0)
    u2 = pop["S"][3:] / np.linalg.norm(pop["S"][3:], axis=0)
    dots = (u1 * u2).sum(0)
    assert stats.kstest(dots, "uniform", args=(-1.0, 2.0)).pvalue > 1e-3


def test_prefix_is_independent_of_the_length_drawn():
    full = P.generate("equal_mass_maxspin_1k")
    part = P.generate("equal_mass_maxspin_1k", 100)
    for k in ("m", "S", "L", "chi"):
        np.testing.assert_array_equal(part[k], full[k][:, :100])
    np.testing.assert_array_equal(part["omega0"], full["omega0"][:100])
    big = P.generate("equal_mass_maxspin_1k", 3000)          # longer than the workload: another draw
    assert big["n"] == 3000 and np.isfinite(big["S"]).all()


def test_workloads_have_distinct_seeds_and_fp32_shares_the_fp64_population():
    seeds = [w.seed for w in P.WORKLOADS.values()]
    a = P.generate("q1to4_1M", 1000)
    b = P.generate("q1to4_1M_fp32split", 1000)
    for k in ("m", "S", "omega0"):
        np.testing.assert_array_equal(a[k], b[k])
    others = [w.seed for w in P.WORKLOADS.values() if w.name not in ("q1to4_1M", "q1to4_1M_fp32split")]
    assert len(set(others)) == len(others) and P.WORKLOADS["q1to4_1M"].seed not in others
    assert len(seeds) == len(P.WORKLOADS)


def test_subset_and_replicate():
    pop = P.generate("adjoint_64k", 50)
    idx = np.array([3, 7, 7, 49])
    sub = P.subset(pop, idx)
    np.testing.assert_array_equal(sub["S"], pop["S"][:, idx])
    assert sub["n"] == 4
    rep = P.replicate(pop, 9)
    assert rep["n"] == 9 and (rep["S"] == pop["S"][:, :1]).all() and (rep["omega0"] == pop["omega0"][0]).all()
