"""pn_integrate_noalloc, the entry point that allocates no device memory
(its persistent launch keeps the work counter and launch descriptor in a
fixed scratch array of the library), against pn_integrate on the same
inputs: two calls in a row on one stream, the second with fewer inspirals,
so the second call must find its counter cleared and its descriptor
rewritten.  Same kernels, so the outputs must agree bit for bit."""
import numpy as np
import pytest

from paper_0908_3889_amd import population as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("y", "t", "steps", "status", "dots")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3889_amd import _lib
    _lib.load()
    yield


def _poisoned(api, n):
    out = api.alloc_outputs(n)
    out["y"].fill_(float("nan"))
    out["t"].fill_(float("nan"))
    out["dots"].fill_(float("nan"))
    out["steps"].fill_(-7)
    out["status"].fill_(-99)
    return out


@pytest.mark.parametrize("precision,schedule", [("fp64", "persistent"), ("fp32split", "persistent"),
                                                ("fp64", "static")])
def test_noalloc_equals_pn_integrate_on_two_calls(precision, schedule):
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M", 3001)           # 47 waves, the last one ragged
    d = api.to_device(pop)
    opts = api.make_opts(precision=precision, schedule=schedule)
    sizes = (3001, 1000)                          # the second call is smaller
    refs = []
    for n in sizes:
        sub = {k: v[..., :n].contiguous() for k, v in d.items()}
        ref = api.pn_integrate(sub["m"], sub["S"], sub["L"], sub["omega0"], pop["omega_f"], pop["tol"], opts)
        torch.cuda.synchronize()
        refs.append({k: v.cpu().numpy() for k, v in ref.items() if k in KEYS})
    # both no-allocation calls queued back to back, then compared
    outs, subs = [], []
    for n in sizes:
        sub = {k: v[..., :n].contiguous() for k, v in d.items()}
        subs.append(sub)
        out = _poisoned(api, n)
        print(f"pn_integrate_noalloc {precision} {schedule} n={n}", flush=True)
        api.pn_integrate_noalloc(sub["m"], sub["S"], sub["L"], sub["omega0"], pop["omega_f"], pop["tol"], out,
                                 opts)
        outs.append(out)
    torch.cuda.synchronize()
    for n, out, ref in zip(sizes, outs, refs):
        assert (ref["status"] == 0).all()
        for k in KEYS:
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k], err_msg=f"n={n}: {k}")


def test_noalloc_argument_checks():
    from paper_0908_3889_amd import _lib, api
    L = _lib.load()
    o = api.make_opts()
    # n > ld, and n beyond the largest size: rejected before any launch
    rc = L.pn_integrate_noalloc(10, 5, None, None, None, None, 0.05, 1e-8, o, None, None, None, None, None, None)
    assert rc == _lib.PN_EINVAL
    rc = L.pn_integrate_noalloc((1 << 36) + 1, (1 << 36) + 1, None, None, None, None, 0.05, 1e-8, o,
                                None, None, None, None, None, None)
    assert rc == _lib.PN_EINVAL
    # n = 0 launches nothing
    rc = L.pn_integrate_noalloc(0, 0, None, None, None, None, 0.05, 1e-8, o, None, None, None, None, None, None)
    assert rc == _lib.PN_OK
