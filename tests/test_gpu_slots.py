"""Call slots of persistent launches under load (the host bookkeeping itself
is tested on the CPU in test_slots.py).

More launches are queued, on two streams, than the ring has slots (1024), so
slots are reused while earlier launches may still be queued or running; a
slot rewritten under a running launch would give wrong outputs without an
error (the silent failure of Sec. III).  A call captured into a graph keeps
a slot of its own, so replaying the graph on one stream while more than
1024 direct calls run on another cannot disturb either.  Every output is
compared bitwise with the eager result of the same call."""
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


KEYS = ("y", "t", "steps", "status", "dots")


def _setup(n=192):
    from paper_0908_3889_amd import api
    pop = P.generate("adjoint_64k", n)          # three waves, short inspirals
    d = api.to_device(pop)
    ref = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    torch.cuda.synchronize()
    return api, pop, d, {k: v.cpu().numpy() for k, v in ref.items()}


def _same(out, ref, what):
    for k in KEYS:
        np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k], err_msg=f"{what}: {k}")


def test_launches_queued_on_two_streams_beyond_the_ring():
    api, pop, d, ref = _setup()
    calls = 600
    outs = [[api.alloc_outputs(pop["n"]) for _ in range(calls)] for _ in range(2)]
    for pair in outs:
        for o in pair:
            o["y"].fill_(float("nan"))
            o["status"].fill_(-99)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i in range(calls):
        for s, pair in zip(streams, outs):
            api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                             out=pair[i], stream=s)
    torch.cuda.synchronize()
    for j, pair in enumerate(outs):
        for i, o in enumerate(pair):
            _same(o, ref, f"stream {j} call {i}")


def test_graph_replays_beside_more_direct_calls_than_the_ring_holds():
    api, pop, d, ref = _setup()
    gout = api.alloc_outputs(pop["n"])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                # warm-up outside the capture
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], out=gout, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], out=gout,
                         stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    calls = 1100
    outs = [api.alloc_outputs(pop["n"]) for _ in range(calls)]
    torch.cuda.synchronize()
    main, rep = torch.cuda.Stream(), torch.cuda.Stream()
    for i in range(calls):
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], out=outs[i],
                         stream=main)
        if i % 100 == 99:
            # a replay on its own stream, overlapping the direct calls; one
            # replay at a time (replays of one graph write the same outputs)
            with torch.cuda.stream(rep):
                g.replay()
            rep.synchronize()
            _same(gout, ref, f"replay after direct call {i}")
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        _same(o, ref, f"direct call {i}")
