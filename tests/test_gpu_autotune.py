"""pn_autotune: it times every candidate launch shape and returns the fastest,
and the shape it returns gives the same integration bit for bit."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("precision", ["fp64", "fp32split"])
def test_autotune_picks_the_fastest_and_changes_nothing_else(precision):
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M", 40000)
    d = api.to_device(pop)
    opts = api.make_opts(precision=precision)
    best, table = api.autotune(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                               sample=20000)
    assert len(table) == 8 and all(v > 0 for v in table.values())
    assert table[(best.refill_min, best.block)] == min(table.values())
    assert best.precision == opts.precision
    a = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts)
    b = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], best)
    torch.cuda.synchronize()
    for k in ("y", "t", "steps", "status", "dots"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), err_msg=k)
