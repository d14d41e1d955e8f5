"""Pins of the statistics oracle (Sec. V) against independent library
routines and closed forms."""
import math

import numpy as np
import pytest
from scipy import stats as st

from oracle import stats as S


def test_histogram_edges_and_exclusions():
    x = np.array([-1.0, -0.9, -0.9 + 1e-17, 0.0, 0.95, 0.9999, 1.0, 1.5, -1.0000001, np.nan])
    h = S.histogram(x, -1.0, 1.0, 20)
    ref = np.zeros(20, np.int64)
    ref[0] = 1            # -1
    ref[1] = 2            # -0.9 (a left edge) and -0.9 + 1e-17 (rounds to it)
    ref[10] = 1           # 0
    ref[19] = 3           # 0.95, 0.9999 and 1 (the last bin is closed)
    np.testing.assert_array_equal(h, ref)


@pytest.mark.parametrize("nbins", [20, 79, 100])
def test_histogram_matches_numpy(nbins):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-1, 1, 100000), S.bin_edges(-1.0, 1.0, nbins)])
    np.testing.assert_array_equal(S.histogram(x, -1.0, 1.0, nbins), np.histogram(x, nbins, (-1.0, 1.0))[0])


def test_histogram2d_matches_numpy():
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, 50000)
    y = np.clip(x + rng.normal(0, 0.2, x.size), -1, 1)
    ref = np.histogram2d(x, y, 79, [[-1.0, 1.0], [-1.0, 1.0]])[0].astype(np.int64)
    np.testing.assert_array_equal(S.histogram2d(x, y, -1.0, 1.0, 79), ref)


def test_pearson_against_scipy_and_closed_forms():
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 200000)
    y = 0.7 * x + rng.normal(0, 0.3, x.size)
    p = S.pearson(x, y)
    assert abs(p["r"] - st.pearsonr(x, y)[0]) < 1e-12
    assert abs(p["std_x"] - np.std(x, ddof=1)) < 1e-14
    assert S.pearson(x, 3.0 * x - 1.0)["r"] == pytest.approx(1.0, abs=1e-14)
    assert S.pearson(x, -2.0 * x)["r"] == pytest.approx(-1.0, abs=1e-14)
    assert abs(S.pearson(x, rng.uniform(-1, 1, x.size))["r"]) < 5 / math.sqrt(x.size)


def test_kde_against_scipy_and_a_single_gaussian():
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, 3000)
    h = S.silverman_bandwidth(x)
    assert h == pytest.approx(1.06 * np.std(x, ddof=1) * x.size ** -0.2, rel=1e-14)
    grid = S.kde_grid(-1.5, 1.5, 61)
    ref = st.gaussian_kde(x, bw_method=1.06 * x.size ** -0.2)(grid)
    np.testing.assert_allclose(S.kde(x, grid, h), ref, rtol=1e-11, atol=0)
    # one point: the normal density of width h; it integrates to 1
    g = S.kde_grid(-2, 2, 4001)
    p = S.kde(np.array([0.3]), g, 0.25)
    np.testing.assert_allclose(p, np.exp(-0.5 * ((g - 0.3) / 0.25) ** 2) / (0.25 * math.sqrt(2 * math.pi)),
                               rtol=1e-14)
    assert np.trapezoid(p, g) == pytest.approx(1.0, abs=1e-9)


@pytest.mark.parametrize("n", [1, 7, 1000, 100000])
def test_ks_against_scipy(n):
    rng = np.random.default_rng(5 + n)
    x = rng.uniform(-1, 1, n)
    k = S.ks_uniform(x, -1.0, 1.0)
    ref = st.kstest(x, "uniform", args=(-1.0, 2.0))
    assert k["D"] == pytest.approx(ref.statistic, rel=1e-14, abs=1e-16)
    assert k["p"] == pytest.approx(st.kstwobign.sf(math.sqrt(n) * k["D"]), rel=1e-9, abs=1e-15)


def test_ks_closed_forms():
    n = 1000
    mid = -1.0 + 2.0 * (np.arange(n) + 0.5) / n          # the evenly spread sample
    assert S.ks_uniform(mid, -1.0, 1.0)["D"] == pytest.approx(0.5 / n, rel=1e-12)
    assert S.ks_uniform(np.full(n, 1.0), -1.0, 1.0)["D"] == pytest.approx(1.0)
    for lam in (0.3, 0.8, 1.0, 1.5, 3.0):
        assert S.kolmogorov_sf(lam) == pytest.approx(st.kstwobign.sf(lam), rel=1e-12, abs=1e-300)
