"""The discrete adjoint (pn_integrate_adjoint) against the oracle.

The adjoint differentiates the Dormand-Prince map with the accepted step
sizes frozen.  The GPU's own recorded step sequence is replayed by the
oracle, so both sides differentiate the same map:
  * the oracle's forward-mode tangent (dual numbers) along random directions
    must satisfy <grad, direction> = <gy, dy_final> + gt dt_final
    (the adjoint/tangent identity), to rounding;
  * central differences of the oracle's replay (h = 1e-6) agree to ~1e-6;
  * the checkpoint spacing K does not change the result.
"""
import numpy as np
import pytest

import oracle
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


def _record(pop, K=16, cap=1024, **kw):
    from paper_0908_3889_amd import api
    d = api.to_device(pop)
    rec = api.pn_integrate_record(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                  api.make_opts(**kw), cap_steps=cap, ckpt_every=K)
    torch.cuda.synchronize()
    return d, rec


def _replay_of(rec):
    tape = rec["tape"].cpu().numpy()
    cap = rec["cap_steps"]
    return {"h": np.ascontiguousarray(tape[:, 2:2 + cap]), "n_t": tape[:, 0].astype(np.int32),
            "n_w": tape[:, 1].astype(np.int32)}


def _adjoint(d, pop, rec, gy, gt, **kw):
    from paper_0908_3889_amd import api
    g = api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, torch.from_numpy(gy).cuda(),
                                 None if gt is None else torch.from_numpy(gt).cuda(), api.make_opts(**kw))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


@pytest.mark.parametrize("workload,n", [("adjoint_64k", 300), ("q1to4_1M", 130), ("batching_4M", 65)])
def test_adjoint_equals_oracle_tangent(workload, n):
    pop = P.generate(workload, n)
    d, rec = _record(pop, K=16, cap=4096)
    st = rec["status"].cpu().numpy()
    assert (st == 0).all()
    replay = _replay_of(rec)
    rng = np.random.default_rng(11)
    gy = rng.normal(size=(10, n))
    gt = rng.normal(size=n) * 1e-5
    g = _adjoint(d, pop, rec, gy, gt)
    dm = rng.normal(size=(2, n)) * 1e-2
    dS = rng.normal(size=(6, n)) * 1e-2
    dL = rng.normal(size=(3, n)) * 1e-2
    dw = rng.normal(size=n) * 1e-5
    tg = oracle.tangent(pop["m"], pop["S"], pop["L"], pop["omega0"], dm, dS, dL, dw, pop["omega_f"],
                        pop["tol"], replay, nthreads=8)
    assert (tg["status"] == 0).all()
    # the oracle replays the GPU's step sequence to the GPU's final state
    yg = rec["y"].cpu().numpy()
    assert np.abs(tg["y"] - yg).max() < 1e-9
    lhs = ((g["m"] * dm).sum(0) + (g["S0"] * dS).sum(0) + (g["L0"] * dL).sum(0) + g["omega0"] * dw)
    rhs = (gy * tg["dy"]).sum(0) + gt * tg["dt"]
    scale = np.abs(g["m"] * dm).sum(0) + np.abs(g["S0"] * dS).sum(0) + np.abs(g["L0"] * dL).sum(0) \
        + np.abs(g["omega0"] * dw) + np.abs(gy * tg["dy"]).sum(0)
    rel = np.abs(lhs - rhs) / scale
    assert rel.max() < 1e-9, (rel.max(), int(rel.argmax()))


def test_adjoint_against_central_differences_of_the_replay():
    n = 12
    pop = P.generate("adjoint_64k", n)
    d, rec = _record(pop, K=16)
    replay = _replay_of(rec)
    rng = np.random.default_rng(5)
    gy = rng.normal(size=(10, n))
    gy[0] = 0.0
    gt = rng.normal(size=n) * 1e-5
    g = _adjoint(d, pop, rec, gy, gt)

    def loss(m, S, L, w):
        r = oracle.integrate(m, S, L, w, pop["omega_f"], pop["tol"], replay=replay, nthreads=8)
        return (gy * r["y"]).sum(0) + gt * r["t"]

    eps = 1e-6
    base = dict(m=pop["m"], S=pop["S"], L=pop["L"], w=pop["omega0"])
    checks = [("m", 2, g["m"]), ("S", 6, g["S0"]), ("L", 3, g["L0"]), ("w", 1, g["omega0"][None])]
    for name, comps, grad in checks:
        for c in range(comps):
            plus = {k: v.copy() for k, v in base.items()}
            minus = {k: v.copy() for k, v in base.items()}
            if name == "w":
                scale_in = pop["omega0"]
                plus["w"] = plus["w"] + eps * scale_in
                minus["w"] = minus["w"] - eps * scale_in
            else:
                scale_in = 1.0
                plus[name][c] += eps
                minus[name][c] -= eps
            fd = (loss(**plus) - loss(**minus)) / (2 * eps)
            ad = grad[c] * scale_in
            assert np.abs(fd - ad).max() < 1e-6 * max(1.0, np.abs(ad).max()), (name, c, fd, ad)


def test_checkpoint_spacing_does_not_change_the_gradient():
    n = 200
    pop = P.generate("adjoint_64k", n)
    rng = np.random.default_rng(3)
    gy = rng.normal(size=(10, n))
    gt = rng.normal(size=n) * 1e-5
    res = []
    for K in (1, 16, 64, 256):
        d, rec = _record(pop, K=K)
        res.append(_adjoint(d, pop, rec, gy, gt))
    for r in res[1:]:
        for k in ("m", "S0", "L0", "omega0"):
            np.testing.assert_allclose(r[k], res[0][k], rtol=1e-10, atol=1e-12 * np.abs(res[0][k]).max())


def test_adjoint_status_handling():
    n = 70
    pop = P.generate("adjoint_64k", n)
    pop["omega0"] = pop["omega0"].copy()
    pop["omega0"][0] = 0.06                       # done at start: identity
    d, rec = _record(pop, K=16)
    st = rec["status"].cpu().numpy()
    assert st[0] == 1 and (st[1:] == 0).all()
    gy = np.random.default_rng(0).normal(size=(10, n))
    g = _adjoint(d, pop, rec, gy, None)
    np.testing.assert_array_equal(g["S0"][:, 0], gy[1:7, 0])
    np.testing.assert_array_equal(g["L0"][:, 0], gy[7:, 0])
    assert g["omega0"][0] == gy[0, 0] and (g["m"][:, 0] == 0).all()
    # a too-small tape ends with TAPE_FULL and a NaN gradient
    d, rec = _record(pop, K=16, cap=20)
    st = rec["status"].cpu().numpy()
    assert (st[1:] == -6).all()
    g = _adjoint(d, pop, rec, gy, None)
    assert np.isnan(g["S0"][:, 1:]).all()


def test_autograd_function_loss_of_the_differentiation_workload():
    """loss = sum_i S1(final).S2(final) + sum_i L_hat_z(final), differentiated
    with respect to the initial spins and masses."""
    from paper_0908_3889_amd import api
    n = 256
    pop = P.generate("adjoint_64k", n)
    d = api.to_device(pop)
    m = d["m"].clone().requires_grad_(True)
    S = d["S"].clone().requires_grad_(True)
    L = d["L"].clone().requires_grad_(True)
    w = d["omega0"].clone().requires_grad_(True)
    y, t, status, steps = api.PNIntegrate.apply(m, S, L, w, pop["omega_f"], pop["tol"], 16, 512)
    loss = (y[1:4] * y[4:7]).sum() + y[9].sum()
    loss.backward()
    torch.cuda.synchronize()
    assert (status == 0).all()
    # the same through the explicit call, with gy = dloss/dy
    yv = y.detach()
    gy = torch.zeros_like(yv)
    gy[1:4] = yv[4:7]
    gy[4:7] = yv[1:4]
    gy[9] = 1.0
    rec = api.pn_integrate_record(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                  cap_steps=512, ckpt_every=16)
    g = api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, gy)
    torch.cuda.synchronize()
    torch.testing.assert_close(S.grad, g["S0"], rtol=1e-12, atol=1e-14)
    torch.testing.assert_close(m.grad, g["m"], rtol=1e-12, atol=1e-14)
    # free (adaptive) finite differences agree only to the controller's O(tol) noise
    i, eps = 3, 1e-6
    Sp = d["S"].clone(); Sp[2, i] += eps
    Sm = d["S"].clone(); Sm[2, i] -= eps
    lp = api.pn_integrate(d["m"], Sp, d["L"], d["omega0"], pop["omega_f"], pop["tol"])["y"]
    lm = api.pn_integrate(d["m"], Sm, d["L"], d["omega0"], pop["omega_f"], pop["tol"])["y"]
    f = lambda yy: float(((yy[1:4] * yy[4:7]).sum(0) + yy[9])[i])
    fd = (f(lp) - f(lm)) / (2 * eps)
    assert abs(fd - float(S.grad[2, i])) < 1e-2 * max(1.0, abs(fd))


def test_record_is_the_same_under_every_launch_shape():
    """The tape (steps and checkpoints) and the gradient do not depend on the
    schedule or the block size of the recording launch."""
    n = 333
    pop = P.generate("batching_4M", n)
    gy = np.random.default_rng(4).normal(size=(10, n))
    K, cap = 16, 4096
    base_d, base = _record(pop, K=K, cap=cap)
    gb = _adjoint(base_d, pop, base, gy, None)

    def written(tape):
        # the counts, the N accepted step sizes and checkpoints 0 .. N // K
        # (the rest of each row is never written)
        out = []
        for row in tape:
            N = int(row[0] + row[1])
            out.append(np.concatenate([row[:2 + N], row[2 + cap:2 + cap + 10 * (N // K + 1)]]))
        return out

    wb = written(base["tape"].cpu().numpy())
    for kw in (dict(schedule="static"), dict(block=64, refill_min=1), dict(block=512)):
        d, rec = _record(pop, K=K, cap=cap, **kw)
        for a, b in zip(written(rec["tape"].cpu().numpy()), wb):
            np.testing.assert_array_equal(a, b, err_msg=str(kw))
        g = _adjoint(d, pop, rec, gy, None)
        for k in ("m", "S0", "L0", "omega0"):
            np.testing.assert_array_equal(g[k], gb[k], err_msg=f"{kw} {k}")


@pytest.mark.parametrize("K", [16, 64, 256])
def test_full_size_adjoint_samples(K):
    """The whole 65,536-inspiral differentiation workload in the benchmark's
    launch configuration (tape cap 1024, lanes ordered by step count, the
    gradient of sum S1.S2 + sum L_hat_z), checked on 64 sampled inspirals
    against the oracle's tangent of the GPU's own step sequence."""
    from paper_0908_3889_amd import api
    pop = P.generate("adjoint_64k")
    n = pop["omega0"].size
    d = api.to_device(pop)
    rec = api.pn_integrate_record(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"],
                                  cap_steps=1024, ckpt_every=K)
    y = rec["y"]
    gy = torch.zeros_like(y)
    gy[1:4] = y[4:7]
    gy[4:7] = y[1:4]
    gy[9] = 1.0
    order = torch.argsort(rec["steps"][0], descending=True).to(torch.int32)
    g = api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, gy, order=order)
    torch.cuda.synchronize()
    assert bool((rec["status"] == 0).all())
    idx = np.sort(np.random.default_rng(K).choice(n, 64, replace=False))
    sub = P.subset(pop, idx)
    tape = rec["tape"].cpu().numpy()[idx]
    replay = {"h": np.ascontiguousarray(tape[:, 2:2 + 1024]), "n_t": tape[:, 0].astype(np.int32),
              "n_w": tape[:, 1].astype(np.int32)}
    rng = np.random.default_rng(K + 1)
    dm, dS, dL = (rng.normal(size=(c, 64)) * 1e-2 for c in (2, 6, 3))
    dw = rng.normal(size=64) * 1e-5
    tg = oracle.tangent(sub["m"], sub["S"], sub["L"], sub["omega0"], dm, dS, dL, dw, pop["omega_f"], pop["tol"],
                        replay, nthreads=8)
    gys = gy.cpu().numpy()[:, idx]
    gg = {k: v.cpu().numpy()[..., idx] for k, v in g.items()}
    lhs = (gg["m"] * dm).sum(0) + (gg["S0"] * dS).sum(0) + (gg["L0"] * dL).sum(0) + gg["omega0"] * dw
    rhs = (gys * tg["dy"]).sum(0)
    scale = np.abs(gg["m"] * dm).sum(0) + np.abs(gg["S0"] * dS).sum(0) + np.abs(gg["L0"] * dL).sum(0) \
        + np.abs(gg["omega0"] * dw) + np.abs(gys * tg["dy"]).sum(0)
    assert (np.abs(lhs - rhs) / scale).max() < 1e-9


def test_bad_tape_rows_and_order_entries_are_refused_per_inspiral():
    """A tape row whose counts are not those of a recorded run gives NaN for
    that inspiral only; order entries outside [0, n) are skipped; the other
    inspirals' gradients are unchanged."""
    from paper_0908_3889_amd import api
    n = 130
    pop = P.generate("adjoint_64k", n)
    d, rec = _record(pop, K=16, cap=1024)
    gy = torch.from_numpy(np.random.default_rng(2).normal(size=(10, n))).cuda()
    ref = {k: v.cpu().numpy() for k, v in api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, gy).items()}
    bad = dict(rec)
    bad["tape"] = rec["tape"].clone()
    bad["tape"][3, 0] = 1.0e9            # more steps than the row holds
    bad["tape"][7, 1] = float("nan")
    bad["tape"][9, 0] = -2.0
    bad["tape"][11, 1] = 2.5
    g = {k: v.cpu().numpy() for k, v in api.pn_integrate_adjoint(d["m"], pop["omega_f"], bad, gy).items()}
    torch.cuda.synchronize()
    rows = [3, 7, 9, 11]
    keep = np.setdiff1d(np.arange(n), rows)
    for k in ("m", "S0", "L0", "omega0"):
        assert np.isnan(g[k][..., rows]).all(), k
        np.testing.assert_array_equal(g[k][..., keep], ref[k][..., keep])
    # an order with two entries out of range: the inspirals they displace get
    # no output, every other one is as without an order
    order = torch.arange(n, dtype=torch.int32, device="cuda")
    order[5] = -1
    order[6] = n
    g = {k: v.cpu().numpy() for k, v in api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, gy,
                                                                    order=order).items()}
    keep = np.setdiff1d(np.arange(n), [5, 6])
    for k in ("m", "S0", "L0", "omega0"):
        np.testing.assert_array_equal(g[k][..., keep], ref[k][..., keep])


def test_central_differences_on_256_samples_of_the_differentiation_workload():
    """The differentiation workload's check: the gradient of
    L = sum S1.S2 + sum L_hat_z (final) against central differences
    (h = 1e-6) of the oracle's replay of the GPU's recorded steps, for every
    input component of 256 inspirals."""
    from paper_0908_3889_amd import api
    n = 256
    pop = P.generate("adjoint_64k", n)
    d, rec = _record(pop, K=64, cap=1024)
    assert bool((rec["status"] == 0).all())
    y = rec["y"]
    gy = torch.zeros_like(y)
    gy[1:4] = y[4:7]
    gy[4:7] = y[1:4]
    gy[9] = 1.0
    g = {k: v.cpu().numpy() for k, v in api.pn_integrate_adjoint(d["m"], pop["omega_f"], rec, gy).items()}
    torch.cuda.synchronize()
    replay = _replay_of(rec)

    def loss(m, S, L, w):
        r = oracle.integrate(m, S, L, w, pop["omega_f"], pop["tol"], replay=replay, nthreads=8)
        yy = r["y"]
        return (yy[1:4] * yy[4:7]).sum(0) + yy[9]

    eps = 1e-6
    base = dict(m=pop["m"], S=pop["S"], L=pop["L"], w=pop["omega0"])
    worst = 0.0
    for name, comps, grad in (("m", 2, g["m"]), ("S", 6, g["S0"]), ("L", 3, g["L0"]), ("w", 1, g["omega0"][None])):
        for c in range(comps):
            plus = {k: v.copy() for k, v in base.items()}
            minus = {k: v.copy() for k, v in base.items()}
            if name == "w":
                step = eps * pop["omega0"]
                plus["w"] = plus["w"] + step
                minus["w"] = minus["w"] - step
                ad = grad[c] * pop["omega0"]
            else:
                plus[name][c] += eps
                minus[name][c] -= eps
                ad = grad[c]
            fd = (loss(**plus) - loss(**minus)) / (2 * eps)
            err = np.abs(fd - ad) / np.maximum(1.0, np.abs(ad))
            worst = max(worst, float(err.max()))
    print(f"adjoint vs central differences, 256 samples x 12 components: max rel err {worst:.2e}")
    assert worst < 1e-6


# ---------------------------------------------------------------------------
# pn_integrate_replay: the map the adjoint differentiates, on the GPU
# ---------------------------------------------------------------------------
def _gpu_replay(pop, rec, m=None, S=None, L=None, w=None, **kw):
    from paper_0908_3889_amd import api
    t = lambda a, b: torch.from_numpy(np.ascontiguousarray(a if a is not None else b)).cuda()
    r = api.pn_integrate_replay(t(m, pop["m"]), t(S, pop["S"]), t(L, pop["L"]), t(w, pop["omega0"]),
                                pop["omega_f"], rec, api.make_opts(**kw))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("workload,n,K", [("adjoint_64k", 300, 16), ("q1to4_1M", 130, 64), ("batching_4M", 65, 1)])
def test_replay_matches_the_oracle_replay_and_the_recorded_run(workload, n, K):
    from helpers import normwise_rel
    pop = P.generate(workload, n)
    d, rec = _record(pop, K=K, cap=4096)
    assert (rec["status"].cpu().numpy() == 0).all()
    r = _gpu_replay(pop, rec)
    ro = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                          replay=_replay_of(rec), nthreads=8)
    e_or = normwise_rel(r["y"], ro["y"], pop["S"])
    e_rec = normwise_rel(r["y"], rec["y"].cpu().numpy(), pop["S"])
    t_or = np.abs(r["t"] / ro["t"] - 1)
    t_rec = np.abs(r["t"] / rec["t"].cpu().numpy() - 1)
    print(f"{workload}: replay vs oracle replay {e_or.max():.2e} (t {t_or.max():.2e}), "
          f"vs recorded run {e_rec.max():.2e} (t {t_rec.max():.2e})")
    assert (r["y"][0] == pop["omega_f"]).all()
    # 1e-12, and on runs beyond 1000 steps 2e-15 per step: two FP64
    # evaluations of the same map differ by roundings that accumulate with
    # the steps (measured: at most 1.2e-15 per step on the 4M workload's
    # adaptive runs of up to 1,575 steps, whose steps are longer than the
    # fixed-step runs' and amplify a rounding of omega through the
    # precession phase)
    steps = rec["steps"].cpu().numpy()[0]
    bound = np.where(steps > 1000, 2e-15 * steps, 1e-12)
    print(f"  per step beyond 1000 steps: {(e_or / steps)[steps > 1000].max() if (steps > 1000).any() else 0:.2e}")
    assert (e_or < bound).all() and (t_or < 1e-12).all()
    assert (e_rec < bound).all() and (t_rec < 1e-12).all()


def test_replay_at_perturbed_inputs_follows_the_oracle_replay():
    from helpers import normwise_rel
    pop = P.generate("adjoint_64k", 200)
    d, rec = _record(pop, K=16)
    rng = np.random.default_rng(8)
    S = pop["S"] * (1 + 1e-3 * rng.normal(size=pop["S"].shape))
    w = pop["omega0"] * (1 + 1e-4 * rng.normal(size=pop["n"]))
    r = _gpu_replay(pop, rec, S=S, w=w)
    ro = oracle.integrate(pop["m"], S, pop["L"], w, pop["omega_f"], pop["tol"], replay=_replay_of(rec), nthreads=8)
    assert normwise_rel(r["y"], ro["y"], S).max() < 1e-12
    assert np.abs(r["t"] / ro["t"] - 1).max() < 1e-12


def test_adjoint_against_central_differences_of_the_gpu_replay():
    """The same check as against the oracle's replay, with both sides of the
    difference quotient evaluated by pn_integrate_replay."""
    n = 64
    pop = P.generate("adjoint_64k", n)
    d, rec = _record(pop, K=16)
    rng = np.random.default_rng(6)
    gy = rng.normal(size=(10, n))
    gy[0] = 0.0
    gt = rng.normal(size=n) * 1e-5
    g = _adjoint(d, pop, rec, gy, gt)

    def loss(**kw):
        r = _gpu_replay(pop, rec, **kw)
        return (gy * r["y"]).sum(0) + gt * r["t"]

    eps = 1e-6
    worst = 0.0
    for name, comps, grad, arr in (("m", 2, g["m"], pop["m"]), ("S", 6, g["S0"], pop["S"]),
                                   ("L", 3, g["L0"], pop["L"]), ("w", 1, g["omega0"][None], pop["omega0"][None])):
        for c in range(comps):
            plus, minus = arr.copy(), arr.copy()
            scale_in = pop["omega0"] if name == "w" else 1.0
            plus[c] = plus[c] + eps * scale_in
            minus[c] = minus[c] - eps * scale_in
            unpack = (lambda a: a[0]) if name == "w" else (lambda a: a)
            fd = (loss(**{name: unpack(plus)}) - loss(**{name: unpack(minus)})) / (2 * eps)
            ad = grad[c] * scale_in
            err = np.abs(fd - ad).max() / max(1.0, np.abs(ad).max())
            worst = max(worst, err)
            assert err < 1e-6, (name, c, err)
    print(f"largest relative FD - adjoint difference {worst:.2e}")


def test_replay_of_a_bad_tape_row_gives_nan():
    pop = P.generate("adjoint_64k", 10)
    pop["omega0"][9] = pop["omega_f"] * 1.2          # done at start: keeps its initial state
    d, rec = _record(pop, K=16)
    assert rec["status"].cpu().numpy()[9] == 1
    rec = dict(rec)
    tape = rec["tape"].clone()
    tape[3, 0] = 0.5                  # not an integer count
    tape[5, 1] = -1.0                 # negative
    tape[7, 0] = float(rec["cap_steps"] + 1)
    rec["tape"] = tape
    r = _gpu_replay(pop, rec)
    bad = [3, 5, 7]
    assert np.isnan(r["y"][:, bad]).all() and np.isnan(r["t"][bad]).all()
    good = np.setdiff1d(np.arange(10), bad)
    assert np.isfinite(r["y"][:, good]).all()
    np.testing.assert_array_equal(r["y"][0, 9], pop["omega0"][9])
    np.testing.assert_array_equal(r["y"][1:7, 9], pop["S"][:, 9])
    assert r["t"][9] == 0.0
