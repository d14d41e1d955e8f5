"""Pins of the oracle's counter-based generator and population draw."""
import numpy as np
import pytest
from scipy import stats as st

from oracle import generate as G


@pytest.mark.parametrize("key,counter", [((0, 0), (1, 0, 0, 0)), ((123, 456), (5, 0, 0, 0)),
                                          ((2 ** 63 + 7, 99), (17, 3, 0, 0)),
                                          ((1, 2), (2 ** 64 - 1, 0, 9, 0))])
def test_philox_block_matches_numpy(key, counter):
    """numpy.random.Philox is Philox4x64-10; its state counter is the block's
    counter minus one (it increments before producing a block)."""
    c = np.array(counter, dtype=np.uint64)
    prev = c.copy()
    if prev[0] == 0:
        prev[0] = np.uint64(2 ** 64 - 1)
        prev[1] -= np.uint64(1)
    else:
        prev[0] -= np.uint64(1)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    ref = bg.random_raw(4)
    got = G.philox4x64([np.array([v], dtype=np.uint64) for v in counter], key)[:, 0]
    np.testing.assert_array_equal(got, ref)


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    hi, lo = G.mulhilo(a, G.M0)
    for x, h, l in zip(a[:200], hi[:200], lo[:200]):
        p = int(x) * int(G.M0)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_uniform_range_and_resolution():
    assert G.uniform(np.array([0], np.uint64))[0] == 0.0
    assert G.uniform(np.array([2 ** 64 - 1], np.uint64))[0] == 1.0 - 2.0 ** -53


def test_population_distributions():
    n = 200000
    p = G.population(n, 42, ("uniform", 1.0, 4.0), ("uniform", 0.0, 1.0), ("fixed", 0.005))
    m1, m2 = p["m"]
    q = m1 / m2
    assert np.allclose(m1 + m2, 1.0, atol=1e-15) and (q >= 1.0).all() and (q <= 4.0 + 1e-12).all()
    assert st.kstest((q - 1.0) / 3.0, "uniform").pvalue > 1e-3
    # spin directions uniform on the sphere: each coordinate of S_hat uniform on [-1, 1]
    s1 = p["S"][:3] / np.linalg.norm(p["S"][:3], axis=0)
    for c in range(3):
        assert st.kstest((s1[c] + 1.0) / 2.0, "uniform").pvalue > 1e-3
    chi1 = np.linalg.norm(p["S"][:3], axis=0) / m1 ** 2
    assert st.kstest(chi1, "uniform").pvalue > 1e-3
    assert (p["L"][2] == 1.0).all() and (p["omega0"] == 0.005).all()


def test_population_streams_are_per_inspiral():
    """Inspiral i depends only on (seed, i): any slice equals the same slice of a
    larger draw, and another seed gives other values."""
    a = G.population(1000, 7, ("fixed", 1.0), ("fixed", 1.0, 1.0), ("fixed", 0.01))
    b = G.population(300, 7, ("fixed", 1.0), ("fixed", 1.0, 1.0), ("fixed", 0.01), first=500)
    np.testing.assert_array_equal(a["S"][:, 500:800], b["S"])
    c = G.population(1000, 8, ("fixed", 1.0), ("fixed", 1.0, 1.0), ("fixed", 0.01))
    assert not np.array_equal(a["S"], c["S"])
