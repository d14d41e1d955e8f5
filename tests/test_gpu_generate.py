"""The on-device population generator against the oracle's draw (bit for
bit), and the streamed K-S run against the same computation unstreamed."""
import numpy as np
import pytest

from oracle import generate as G
from oracle import stats as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3889_amd import _lib
    _lib.load()
    yield


SPECS = [
    (dict(q=(1.0, 4.0), chi1=(0.0, 1.0), chi2=(0.0, 1.0), omega0=(0.005, 0.005), seed=9083889),
     (("uniform", 1.0, 4.0), ("uniform", 0.0, 1.0), ("fixed", 0.005))),
    (dict(q=(1.0, 1.0), chi1=(0.7, 0.7), chi2=(0.7, 0.7), omega0=(0.004, 0.006), seed=2 ** 63 + 11),
     (("fixed", 1.0), ("fixed", 0.7, 0.7), ("uniform", 0.004, 0.006))),
]


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("first,n", [(0, 100003), (12345, 777)])
def test_generate_bit_exact(k, first, n):
    from paper_0908_3889_amd import api
    kw, ospec = SPECS[k]
    got = api.pn_generate(n, api.gen_spec(**kw), first)
    ref = G.population(n, kw["seed"], *ospec, first=first)
    for key in ("m", "S", "L", "omega0"):
        np.testing.assert_array_equal(got[key].cpu().numpy(), ref[key], err_msg=key)


def test_generate_leading_dimension_and_arguments():
    from paper_0908_3889_amd import _lib, api
    kw, ospec = SPECS[0]
    n, ld = 1000, 1024
    buf = {k: torch.full((c, ld), 7.0, dtype=torch.float64, device="cuda") for k, c in (("m", 2), ("S", 6), ("L", 3))}
    out = {k: v[:, :n] for k, v in buf.items()}
    out["omega0"] = torch.empty(n, dtype=torch.float64, device="cuda")
    api.pn_generate(n, api.gen_spec(**kw), 0, out=out)
    ref = G.population(n, kw["seed"], *ospec)
    np.testing.assert_array_equal(buf["S"][:, :n].cpu().numpy(), ref["S"])
    assert (buf["S"][:, n:] == 7.0).all()
    bad = api.gen_spec(q=(0.0, 1.0))
    with pytest.raises(_lib.PnError):
        api.pn_generate(10, bad)
    with pytest.raises(_lib.PnError):
        api.pn_generate(10, api.gen_spec(chi1=(0.5, 1.5)))


def test_streamed_ks_run_equals_the_unstreamed_computation():
    from paper_0908_3889_amd import api
    spec = api.gen_spec(q=(1.0, 1.0), chi1=(0.7, 0.7), chi2=(0.7, 0.7), omega0=(0.01, 0.01), seed=5)
    total = 50000
    res = api.ks_run(total, spec, 0.05, 1e-8, chunk=16384)     # 4 chunks, the last ragged
    torch.cuda.synchronize()
    assert int(res["not_ok"]) == 0
    pop = api.pn_generate(total, spec)
    out = api.pn_integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], 0.05, 1e-8)
    x = out["dots"][0].cpu().numpy()
    np.testing.assert_array_equal(res["final_s1s2"].cpu().numpy(), x)
    ks = S.ks_uniform(x, -1.0, 1.0)
    assert res["ks"][0].item() == ks["D"]
    assert res["ks"][1].item() == pytest.approx(ks["p"], rel=1e-12, abs=1e-300)
    np.testing.assert_array_equal(res["hist"].cpu().numpy(), S.histogram(x, -1.0, 1.0, 100))
