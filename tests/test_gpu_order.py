"""The longest-first hand-out order (pn_cost_order) and pn_opts.order.

pn_cost_order must return a permutation of 0..n-1 sorted by its cost key
(checked against the same leading-order estimate written here in numpy);
integrating in any order must give every inspiral bit-identical outputs
(the order only changes which lane takes which inspiral when); entries
outside [0, n) are skipped and the inspirals they leave out keep their
outputs untouched."""
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


def cost_key(pop):
    """The estimate of pn_cost_order: the larger over the two spins of
    (4 + 3 m_j/m_i) (1/omega0 - 1/omega_f)/M times the 1/5 power of the spin's
    component normal to the initial total angular momentum."""
    m1, m2 = pop["m"]
    S1, S2, Lh, w0, wf = pop["S"][:3], pop["S"][3:], pop["L"], pop["omega0"], pop["omega_f"]
    M = m1 + m2
    eta = m1 * m2 / M**2
    J = eta * M**(5 / 3) * w0**(-1 / 3) * Lh + S1 + S2
    Jh = J / np.linalg.norm(J, axis=0)

    def normal(v):
        va = (v * Jh).sum(0)
        return np.sqrt(np.maximum((v * v).sum(0) - va * va, 0.0))
    span = (1 / w0 - 1 / wf) / M
    return span * np.maximum((4 + 3 * m2 / m1) * normal(S1)**0.2, (4 + 3 * m1 / m2) * normal(S2)**0.2)


@pytest.mark.parametrize("workload,n", [("q1to4_1M", 5003), ("batching_4M", 4099), ("q1to4_1M", 1 << 20)])
def test_cost_order_is_a_sorted_permutation(workload, n):
    from paper_0908_3889_amd import api
    pop = P.generate(workload, n)
    d = api.to_device(pop)
    print(f"pn_cost_order {workload} n={n}", flush=True)
    order = api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"])
    torch.cuda.synchronize()
    o = order.cpu().numpy()
    print(f"unique {np.unique(o).size} min {o.min()} max {o.max()}", flush=True)
    np.testing.assert_array_equal(np.sort(o), np.arange(n))
    key = cost_key(pop)
    k = key[o]
    # sorted by the key's upper 16 float bits (7 mantissa bits): each key is
    # at most 1 % above every key before it
    run_min = np.minimum.accumulate(k)
    assert (k <= run_min * 1.01).all()
    assert np.corrcoef(np.arange(n), -k)[0, 1] > 0.9


def test_done_at_start_and_bad_inputs_come_last():
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M", 1000)
    pop["omega0"][[3, 500]] = pop["omega_f"] * 1.5        # done at start
    pop["m"][0, 7] = -1.0                                 # refused
    d = api.to_device(pop)
    o = api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"]).cpu().numpy()
    assert sorted(o[-3:].tolist()) == [3, 7, 500]


@pytest.mark.parametrize("precision,schedule", [("fp64", "persistent"), ("fp32split", "persistent"),
                                                ("fp64", "static")])
def test_results_do_not_depend_on_the_order(precision, schedule):
    from paper_0908_3889_amd import api
    pop = P.generate("batching_4M", 3001)
    d = api.to_device(pop)
    ref = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                           api.make_opts(precision=precision, schedule=schedule))
    rng = np.random.default_rng(5)
    orders = {"cost": api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"]),
              "random": torch.from_numpy(rng.permutation(pop["n"]).astype(np.int32)).cuda()}
    for name, order in orders.items():
        out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                               api.make_opts(precision=precision, schedule=schedule, order=order))
        torch.cuda.synchronize()
        for k in KEYS:
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=f"{name}: {k}")


def test_entries_outside_the_range_are_skipped():
    from paper_0908_3889_amd import api
    pop = P.generate("adjoint_64k", 700)
    d = api.to_device(pop)
    ref = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"])
    o = np.arange(pop["n"], dtype=np.int32)
    o[[10, 300]] = [-5, pop["n"] + 9]                 # inspirals 10 and 300 are left out
    for schedule in ("persistent", "static"):
        out = api.alloc_outputs(pop["n"])
        out["status"].fill_(-99)
        api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                         api.make_opts(schedule=schedule, order=torch.from_numpy(o).cuda()), out=out)
        torch.cuda.synchronize()
        st = out["status"].cpu().numpy()
        assert (st[[10, 300]] == -99).all()
        keep = np.ones(pop["n"], bool)
        keep[[10, 300]] = False
        np.testing.assert_array_equal(out["y"].cpu().numpy()[:, keep], ref["y"].cpu().numpy()[:, keep])
        np.testing.assert_array_equal(st[keep], ref["status"].cpu().numpy()[keep])


def test_packed_records_hold_the_inputs():
    """pn_cost_order's packed output: per inspiral m1, m2, omega0, S1, S2,
    L_hat and four zeros, bit for bit, on a size that is not a multiple of
    the block (and with a bad input and one done at start)."""
    from paper_0908_3889_amd import api
    pop = P.generate("q1to4_1M", 5003)
    pop["omega0"] = pop["omega0"].copy(); pop["m"] = pop["m"].copy()
    pop["omega0"][7] = 0.06
    pop["m"][1, 11] = 0.0
    d = api.to_device(pop)
    packed = api.packed_inputs(pop["n"])
    packed.fill_(float("nan"))
    api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], packed=packed)
    torch.cuda.synchronize()
    got = packed.cpu().numpy()
    want = np.concatenate([pop["m"], pop["omega0"][None], pop["S"], pop["L"], np.zeros((4, pop["n"]))]).T
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("precision", ["fp64", "fp32split", "fp32"])
def test_packed_inputs_give_the_same_results(precision):
    """Reading the inputs from the packed records (with the cost order, in
    index order, the static schedule, the phase kernel and the no-allocation
    entry point) gives every inspiral the bits of the SoA run."""
    from paper_0908_3889_amd import api
    pop = P.generate("batching_4M", 3001)
    pop["omega0"] = pop["omega0"].copy(); pop["S"] = pop["S"].copy()
    pop["omega0"][5] = 0.06                   # done at start
    pop["S"][2, 9] = np.nan                   # bad input
    d = api.to_device(pop)
    ref = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                           api.make_opts(precision=precision))
    packed = api.packed_inputs(pop["n"])
    order = api.pn_cost_order(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], packed=packed)
    runs = {"cost order": api.make_opts(precision=precision, order=order, packed=packed),
            "index order": api.make_opts(precision=precision, packed=packed),
            "static": api.make_opts(precision=precision, schedule="static", packed=packed)}
    for name, opts in runs.items():
        out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts)
        torch.cuda.synchronize()
        for k in KEYS:
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=f"{name}: {k}")
    assert ref["status"][5].item() == 1 and ref["status"][9].item() == -4
    ph_ref = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                    api.make_opts(precision=precision))
    ph = api.pn_integrate_phase(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                api.make_opts(precision=precision, order=order, packed=packed))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ph["phase"].cpu().numpy(), ph_ref["phase"].cpu().numpy())
    if precision == "fp64":
        out = api.alloc_outputs(pop["n"])
        api.pn_integrate_noalloc(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], out,
                                 api.make_opts(order=order, packed=packed))
        torch.cuda.synchronize()
        for k in KEYS:
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=f"noalloc: {k}")
