"""The statistics stage (Sec. V) on the GPU against the oracle.

Histogram counts are integers and must agree exactly (the bin decision is
taken against the same FP64 edges on both sides); the moments, the KDE and
the K-S statistic are sums over the sample, compared within bounds derived
from their length."""
import numpy as np
import pytest

from oracle import stats as S
from paper_0908_3889_amd import population as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3889_amd import _lib
    _lib.load()
    yield


def _api():
    from paper_0908_3889_amd import api
    return api


def _sample(n, ncomp=3, seed=0, edges=True):
    """Values on [-1, 1] with bin edges, the ends, out-of-range values and a NaN
    mixed in (the histograms must ignore the last two)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (ncomp, n))
    if edges and n > 400:
        for c in range(ncomp):
            e = S.bin_edges(-1.0, 1.0, 100)
            x[c, :e.size] = e
            x[c, e.size:e.size + 4] = [1.0, -1.0, 1.0000000001, -3.0]
            x[c, e.size + 4] = np.nan
    return x


@pytest.mark.parametrize("nbins", [1, 20, 79, 100, 4096])
def test_histogram_bit_exact(nbins):
    api = _api()
    x = _sample(300007, seed=nbins)
    got = api.pn_histogram(torch.from_numpy(x).cuda(), nbins).cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(got[c], S.histogram(x[c], -1.0, 1.0, nbins))


def test_histogram_leading_dimension_and_other_range():
    api = _api()
    x = _sample(10000, seed=3)
    big = np.full((3, 10240), 7.0)
    big[:, :10000] = x
    t = torch.from_numpy(big).cuda()[:, :10000]
    got = api.pn_histogram(t, 50, lo=-0.5, hi=0.75).cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(got[c], S.histogram(x[c], -0.5, 0.75, 50))


@pytest.mark.parametrize("nbins", [79, 128])
def test_histogram2d_bit_exact(nbins):
    api = _api()
    x = _sample(200003, seed=5)
    y = np.clip(x + np.random.default_rng(6).normal(0, 0.1, x.shape), -1.2, 1.2)
    got = api.pn_histogram2d(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), nbins).cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(got[c], S.histogram2d(x[c], y[c], -1.0, 1.0, nbins))


def test_pearson_against_oracle():
    api = _api()
    rng = np.random.default_rng(8)
    n = 400009
    x = rng.uniform(-1, 1, (3, n))
    y = np.stack([0.9 * x[0] + 0.1 * rng.normal(size=n), -x[1] + 0.5, rng.uniform(-1, 1, n)])
    got = api.pn_pearson(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
    for c in range(3):
        ref = S.pearson(x[c], y[c])
        want = [ref["mean_x"], ref["mean_y"], ref["std_x"], ref["std_y"], ref["r"]]
        # sums of n terms in another order: the deviations to a few hundred ulps;
        # r to 1e-12 absolute (its numerator cancels when r is small)
        np.testing.assert_allclose(got[c, 2:4], want[2:4], rtol=1e-12)
        np.testing.assert_allclose(got[c, :2], want[:2], rtol=0, atol=1e-15)
        assert abs(got[c, 4] - want[4]) < 1e-12
    assert got[1, 4] == pytest.approx(-1.0, abs=1e-14)


def test_kde_against_oracle():
    api = _api()
    x = _sample(30011, seed=9, edges=False)
    xt = torch.from_numpy(x).cuda()
    p = api.pn_pearson(xt, xt)
    sig = p[:, 2].contiguous()
    got = api.pn_kde(xt, sig, 201).cpu().numpy()
    grid = S.kde_grid(-1.0, 1.0, 201)
    for c in range(3):
        ref = S.kde(x[c], grid, S.silverman_bandwidth(x[c]))
        np.testing.assert_allclose(got[c], ref, rtol=1e-11)
    # more grid points than a block has threads, another range
    got = api.pn_kde(xt[:1], sig[:1].contiguous(), 700, lo=-1.5, hi=1.2).cpu().numpy()
    ref = S.kde(x[0], S.kde_grid(-1.5, 1.2, 700), S.silverman_bandwidth(x[0]))
    np.testing.assert_allclose(got[0], ref, rtol=1e-11, atol=1e-300)


@pytest.mark.parametrize("n", [1, 2, 513, 131073])
def test_ks_against_oracle(n):
    api = _api()
    rng = np.random.default_rng(n)
    x = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n) ** 3, np.clip(rng.normal(0, 0.5, n), -1, 1)])
    got = api.pn_ks_uniform(torch.from_numpy(x).cuda()).cpu().numpy()
    for c in range(3):
        ref = S.ks_uniform(x[c], -1.0, 1.0)
        assert got[c, 0] == ref["D"]
        assert got[c, 1] == pytest.approx(ref["p"], rel=1e-12, abs=1e-300)


def test_empty_and_single():
    api = _api()
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    assert (api.pn_histogram(e, 20) == 0).all()
    assert (api.pn_histogram2d(e, e, 10) == 0).all()
    assert torch.isnan(api.pn_pearson(e, e)).all()
    assert torch.isnan(api.pn_ks_uniform(e)).all()
    one = torch.tensor([[0.25], [-0.5], [1.0]], dtype=torch.float64, device="cuda")
    p = api.pn_pearson(one, one).cpu().numpy()
    np.testing.assert_array_equal(p[:, 0], [0.25, -0.5, 1.0])
    assert np.isnan(p[:, 2:]).all()
    ks = api.pn_ks_uniform(one).cpu().numpy()
    for c, v in enumerate([0.25, -0.5, 1.0]):
        assert ks[c, 0] == S.ks_uniform(np.array([v]), -1.0, 1.0)["D"]


def test_statistics_of_the_paper_equal_mass_population():
    """The whole stage on the GPU's own integration of the Sec. V A population:
    identical to the oracle's statistics of the same values, and the paper's
    correlations r = 0.99 (S1.S2) and 0.65 (S_i.L)."""
    api = _api()
    pop = P.generate("paper_equal_mass")
    d = api.to_device(pop)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    y0 = torch.cat([d["omega0"][None], d["S"], d["L"]], 0).contiguous()
    init = api.pn_observables(y0)
    st = api.statistics(init, out["dots"])
    torch.cuda.synchronize()
    xi, xf = init.cpu().numpy(), out["dots"].cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(st["hist"][c].cpu().numpy(), S.histogram(xf[c], -1.0, 1.0, 20))
        np.testing.assert_array_equal(st["hist2d"][c].cpu().numpy(), S.histogram2d(xi[c], xf[c], -1.0, 1.0, 79))
        ref = S.pearson(xi[c], xf[c])
        assert st["pearson"][c, 4].item() == pytest.approx(ref["r"], rel=1e-12)
        kde = S.kde(xf[c], S.kde_grid(-1.0, 1.0, 201), S.silverman_bandwidth(xf[c]))
        np.testing.assert_allclose(st["kde"][c].cpu().numpy(), kde, rtol=1e-11)
        ks = S.ks_uniform(xf[c], -1.0, 1.0)
        assert st["ks"][c, 0].item() == ks["D"]
    r = st["pearson"][:, 4].cpu().numpy()
    assert abs(r[0] - 0.99) < 0.01 and abs(r[1] - 0.65) < 0.03 and abs(r[2] - 0.65) < 0.03


def test_kde_of_final_spin_product_converges_to_uniform():
    """The figure of Sec. V on the kernel density estimate of the final
    S1_hat.S2_hat: as N grows the estimate approaches the uniform density 1/2
    on [-1, 1].  GPU integration of N = 100,000 inspirals of the Sec. V A
    set-up, pn_kde on prefixes of 1,000, 10,000 and 100,000 (Silverman's
    bandwidth from pn_pearson's standard deviation): away from the ends
    (|x| <= 0.8, where the estimate's boundary bias lives) the mean deviation
    from 1/2 shrinks with N (oracle on the same population: 0.029, 0.0099,
    0.0059; largest 0.081, 0.026, 0.017), and each estimate equals the
    oracle's KDE of the same values."""
    api = _api()
    pop = P.generate("paper_equal_mass", 100000)
    d = api.to_device(pop)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    torch.cuda.synchronize()
    assert (out["status"] == 0).all()
    g = S.kde_grid(-1.0, 1.0, 201)
    inner = np.abs(g) <= 0.8
    means, maxes = [], []
    for N in (1000, 10000, 100000):
        x = out["dots"][0:1, :N].contiguous()
        p = api.pn_pearson(x, x)
        kde = api.pn_kde(x, p[:, 2].contiguous()).cpu().numpy()[0]
        xf = x.cpu().numpy()[0]
        np.testing.assert_allclose(kde, S.kde(xf, g, S.silverman_bandwidth(xf)), rtol=1e-11)
        dev = np.abs(kde[inner] - 0.5)
        means.append(dev.mean()); maxes.append(dev.max())
    print("KDE deviation from 1/2 (mean, max) at N = 1e3, 1e4, 1e5:", means, maxes)
    assert means[0] > means[1] > means[2] and means[2] < 0.01
    assert maxes[2] < 0.03


def test_statistics_full_size_workload():
    """The statistics stage over the whole 1M workload's GPU dot products
    (the benchmark's --stats input), against the oracle's statistics of the
    same values."""
    api = _api()
    pop = P.generate("q1to4_1M")
    d = api.to_device(pop)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    y0 = torch.cat([d["omega0"][None], d["S"], d["L"]], 0).contiguous()
    init = api.pn_observables(y0)
    st = api.statistics(init, out["dots"])
    torch.cuda.synchronize()
    xi, xf = init.cpu().numpy(), out["dots"].cpu().numpy()
    h100 = api.pn_histogram(out["dots"], 100).cpu().numpy()
    grid = S.kde_grid(-1.0, 1.0, 201)
    for c in range(3):
        np.testing.assert_array_equal(st["hist"][c].cpu().numpy(), S.histogram(xf[c], -1.0, 1.0, 20))
        np.testing.assert_array_equal(h100[c], S.histogram(xf[c], -1.0, 1.0, 100))
        np.testing.assert_array_equal(st["hist2d"][c].cpu().numpy(), S.histogram2d(xi[c], xf[c], -1.0, 1.0, 79))
        ref = S.pearson(xi[c], xf[c])
        assert st["pearson"][c, 4].item() == pytest.approx(ref["r"], rel=1e-12)
        np.testing.assert_allclose(st["kde"][c].cpu().numpy(), S.kde(xf[c], grid, S.silverman_bandwidth(xf[c])),
                                   rtol=1e-11)
        ks = S.ks_uniform(xf[c], -1.0, 1.0)
        assert st["ks"][c, 0].item() == ks["D"]
        assert st["ks"][c, 1].item() == pytest.approx(ks["p"], rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("ncomp", [1, 7, 16])
def test_many_components(ncomp):
    """Every statistic over up to the largest number of components a call
    takes, each component its own distribution."""
    api = _api()
    rng = np.random.default_rng(ncomp)
    n = 50021
    x = np.stack([np.clip(rng.normal(-0.5 + c / ncomp, 0.2 + 0.02 * c, n), -1, 1) for c in range(ncomp)])
    y = np.stack([0.5 * x[c] + 0.5 * rng.uniform(-1, 1, n) for c in range(ncomp)])
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    h = api.pn_histogram(xt, 37).cpu().numpy()
    h2 = api.pn_histogram2d(xt, yt, 23).cpu().numpy()
    p = api.pn_pearson(xt, yt).cpu().numpy()
    ks = api.pn_ks_uniform(xt).cpu().numpy()
    kde = api.pn_kde(xt, api.pn_pearson(xt, xt)[:, 2].contiguous(), 64).cpu().numpy()
    grid = S.kde_grid(-1.0, 1.0, 64)
    for c in range(ncomp):
        np.testing.assert_array_equal(h[c], S.histogram(x[c], -1.0, 1.0, 37))
        np.testing.assert_array_equal(h2[c], S.histogram2d(x[c], y[c], -1.0, 1.0, 23))
        assert abs(p[c, 4] - S.pearson(x[c], y[c])["r"]) < 1e-12
        ref = S.ks_uniform(x[c], -1.0, 1.0)
        assert ks[c, 0] == ref["D"]
        np.testing.assert_allclose(kde[c], S.kde(x[c], grid, S.silverman_bandwidth(x[c])), rtol=1e-11, atol=1e-300)


def test_too_many_components_is_refused():
    api = _api()
    x = torch.zeros((17, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        api.pn_histogram(x, 10)
