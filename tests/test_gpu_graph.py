"""pn_integrate captured in a HIP graph and replayed.

The counter reset is a kernel (no memset node), so a captured call replays
correctly; each replay is checked bitwise against the eager result, with the
program's own eager work and synchronisations between replays."""
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
def test_pn_integrate_replays_in_a_graph(precision):
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M", 6000)
    d = api.to_device(pop)
    opts = api.make_opts(precision=precision)
    ref = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}

    out = api.alloc_outputs(pop["n"])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):            # warm-up outside the capture
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                         out=out, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts,
                         out=out, stream=torch.cuda.current_stream())
    for rep in range(3):
        # eager work between replays: poison the outputs
        out["y"].fill_(float("nan"))
        out["status"].fill_(-99)
        out["steps"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("y", "t", "steps", "status", "dots"):
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k], err_msg=f"replay {rep} {k}")
