"""Shared helpers for the tests: running the oracle and the GPU path on the
same seeded inputs, and the parity measures."""
import numpy as np

import oracle


def state0(pop):
    return np.concatenate([pop["omega0"][None], pop["S"], pop["L"]])


def normwise_rel(y_a, y_b, S0):
    """Per inspiral, max over the groups of ||a - b|| / scale: omega scaled by
    |omega|, S_i by |S_i(0)| (1 if zero), L_hat by 1."""
    w = np.abs(y_a[0] - y_b[0]) / np.maximum(np.abs(y_b[0]), 1e-300)
    n1 = np.linalg.norm(S0[:3], axis=0); n1[n1 == 0] = 1.0
    n2 = np.linalg.norm(S0[3:], axis=0); n2[n2 == 0] = 1.0
    s1 = np.linalg.norm(y_a[1:4] - y_b[1:4], axis=0) / n1
    s2 = np.linalg.norm(y_a[4:7] - y_b[4:7], axis=0) / n2
    l = np.linalg.norm(y_a[7:10] - y_b[7:10], axis=0)
    return np.max(np.stack([w, s1, s2, l]), axis=0)


def run_oracle(pop, nthreads=0, **kw):
    r = oracle.integrate(pop["m"], pop["S"], pop["L"], pop["omega0"], pop["omega_f"], pop["tol"],
                         nthreads=nthreads, **kw)
    r["dots"] = oracle.observables(r["y"])
    return r


def run_gpu(pop, **kw):
    import torch

    from paper_0908_3889_amd import api
    d = api.to_device(pop)
    opts = api.make_opts(**kw)
    out = api.pn_integrate(d["m"], d["S"], d["L"], d["omega0"], pop["omega_f"], pop["tol"], opts)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
