"""CPU oracle of the statistics the paper computes over the final states
(Sec. V): equal-width histograms, bivariate histograms, the Pearson
product-moment coefficient, the Gaussian kernel density estimator with
Silverman's bandwidth, and the Kolmogorov-Smirnov statistic against the
uniform distribution.

TEST INFRASTRUCTURE, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU baseline use it.  Plain numpy in float64,
written from the definitions, with no blocking or reordering beyond them; it
shares nothing with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np


def bin_edges(lo: float, hi: float, nbins: int) -> np.ndarray:
    """The nbins + 1 edges of equal-width bins on [lo, hi]: lo + i (hi - lo)/nbins,
    the last one exactly hi."""
    step = (hi - lo) / nbins
    e = np.arange(nbins + 1, dtype=np.float64) * step + lo
    e[-1] = hi
    return e


def histogram(x: np.ndarray, lo: float, hi: float, nbins: int) -> np.ndarray:
    """Counts of x in bins [e_i, e_{i+1}) (the last bin closed), values outside
    [lo, hi] and NaN not counted (Sec. V, the histograms of Figs. 2 and 3)."""
    e = bin_edges(lo, hi, nbins)
    x = np.asarray(x, dtype=np.float64)
    keep = (x >= lo) & (x <= hi)
    idx = np.searchsorted(e, x[keep], side="right") - 1
    idx[idx == nbins] = nbins - 1
    return np.bincount(idx, minlength=nbins).astype(np.int64)


def histogram2d(x: np.ndarray, y: np.ndarray, lo: float, hi: float, nbins: int) -> np.ndarray:
    """Bivariate counts [nbins (x), nbins (y)] with the bins of `histogram` in
    each dimension (Sec. V, Figs. 4 and 5: initial against final value)."""
    e = bin_edges(lo, hi, nbins)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    keep = (x >= lo) & (x <= hi) & (y >= lo) & (y <= hi)
    ix = np.searchsorted(e, x[keep], side="right") - 1
    iy = np.searchsorted(e, y[keep], side="right") - 1
    ix[ix == nbins] = nbins - 1
    iy[iy == nbins] = nbins - 1
    return np.bincount(ix * nbins + iy, minlength=nbins * nbins).reshape(nbins, nbins).astype(np.int64)


def pearson(x: np.ndarray, y: np.ndarray) -> dict:
    """Means, standard deviations (with 1/(N-1)) and the Pearson coefficient
    r = 1/(N-1) sum ((x - xbar)/sigma_x)((y - ybar)/sigma_y) (Sec. V)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    mx = x.sum() / n
    my = y.sum() / n
    dx = x - mx
    dy = y - my
    sxx = (dx * dx).sum()
    syy = (dy * dy).sum()
    sxy = (dx * dy).sum()
    return {"mean_x": mx, "mean_y": my, "std_x": math.sqrt(sxx / (n - 1)), "std_y": math.sqrt(syy / (n - 1)),
            "r": sxy / math.sqrt(sxx * syy)}


def silverman_bandwidth(x: np.ndarray) -> float:
    """h = 1.06 sigma N^(-1/5), sigma the standard deviation (Sec. V)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    m = x.sum() / n
    sigma = math.sqrt(((x - m) ** 2).sum() / (n - 1))
    return 1.06 * sigma * n ** -0.2


def kde_grid(lo: float, hi: float, ngrid: int) -> np.ndarray:
    """ngrid evaluation points lo + g (hi - lo)/(ngrid - 1)."""
    return lo + np.arange(ngrid, dtype=np.float64) * ((hi - lo) / (ngrid - 1))


def kde(x: np.ndarray, grid: np.ndarray, h: float) -> np.ndarray:
    """p(x_g) = 1/(N h) sum_j K((x_g - x_j)/h), K(u) = exp(-u^2/2)/sqrt(2 pi)
    (Sec. V), term by term."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(grid.size)
    norm = 1.0 / (x.size * h * math.sqrt(2.0 * math.pi))
    for g, xg in enumerate(grid):
        u = (xg - x) / h
        out[g] = np.exp(-0.5 * u * u).sum() * norm
    return out


def kolmogorov_sf(lam: float) -> float:
    """P(K > lam) for the Kolmogorov distribution: the alternating series
    2 sum_k (-1)^(k-1) exp(-2 k^2 lam^2) for lam >= 1, else one minus the
    theta-function form sqrt(2 pi)/lam sum_k exp(-(2k-1)^2 pi^2 / (8 lam^2))."""
    if lam <= 0.0:
        return 1.0
    if lam >= 1.0:
        s = 0.0
        for k in range(1, 101):
            s += 2.0 * (-1.0) ** (k - 1) * math.exp(-2.0 * k * k * lam * lam)
        return min(1.0, max(0.0, s))
    c = 0.0
    for k in range(1, 101):
        c += math.exp(-((2 * k - 1) ** 2) * math.pi ** 2 / (8.0 * lam * lam))
    return min(1.0, max(0.0, 1.0 - math.sqrt(2.0 * math.pi) / lam * c))


def ks_uniform(x: np.ndarray, lo: float, hi: float) -> dict:
    """Kolmogorov-Smirnov statistic of x against the uniform distribution on
    [lo, hi]: D = max_i max(i/N - F(x_(i)), F(x_(i)) - (i-1)/N) over the sorted
    sample, F(x) = (x - lo)/(hi - lo), and the asymptotic p-value
    P(K > sqrt(N) D) (Sec. V: the K-S test of the final dot products)."""
    xs = np.sort(np.asarray(x, dtype=np.float64))
    n = xs.size
    F = (xs - lo) / (hi - lo)
    i = np.arange(1, n + 1, dtype=np.float64)
    d = max(float((i / n - F).max()), float((F - (i - 1) / n).max()))
    return {"D": d, "p": kolmogorov_sf(math.sqrt(n) * d)}
