"""Seeded synthetic populations of binary-black-hole initial data.

This module only draws inputs. It holds none of the integration method's
arithmetic, and it is the one module that both the GPU path and the CPU
oracle take their inputs from.

What is drawn (paper, Sec. II and Sec. V):

* total mass M = m1 + m2 = 1, since the problem is scale free (Sec. II);
  the mass ratio q = m1/m2 >= 1 gives m1 = q/(1+q), m2 = 1/(1+q);
* spin vectors S_i = chi_i m_i^2 S_hat_i with chi_i in [0, 1] the Kerr
  parameter (Sec. II, just after Eq. (4));
* the spin directions S_hat_i uniform on the unit sphere, drawn with
  Marsaglia's (1972) rejection method, as the paper does (Sec. V);
* the orbital angular momentum direction L_hat = (0, 0, 1), which the paper
  takes without loss of generality (Sec. V);
* the initial orbital frequency omega0 (fixed or log-uniform).

Draw order from one numpy PCG64 stream: q (if random), chi_1 then chi_2
(if random), S_hat_1 then S_hat_2 (Marsaglia), omega0 (if random).

Layout (structure of arrays, float64, C-contiguous):
  m      [2, n]  (m1, m2)
  S      [6, n]  (S1x, S1y, S1z, S2x, S2y, S2z)
  L      [3, n]  (Lx, Ly, Lz)
  omega0 [n]
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 9083889


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: sizes, distributions and tolerances."""
    name: str
    n: int
    q: tuple            # ("fixed", q) or ("uniform", lo, hi)
    chi: tuple          # ("fixed", chi1, chi2) or ("uniform", lo, hi)
    omega0: tuple       # ("fixed", w0) or ("loguniform", lo, hi)
    omega_f: float
    tol: float
    seed: int
    precision: str = "fp64"
    notes: str = field(default="")


# The workloads.  Index k uses seed BASE_SEED + k.
WORKLOADS = {
    "equal_mass_maxspin_1k": Workload(
        "equal_mass_maxspin_1k", 1024, ("fixed", 1.0), ("fixed", 1.0, 1.0),
        ("fixed", 0.01), 0.05, 1e-10, BASE_SEED + 0,
        notes="m1=m2=0.5, chi=1, isotropic spins, omega 0.01 -> 0.05, tol 1e-10"),
    "q1to4_1M": Workload(
        "q1to4_1M", 1 << 20, ("uniform", 1.0, 4.0), ("uniform", 0.0, 1.0),
        ("fixed", 0.005), 0.05, 1e-8, BASE_SEED + 1,
        notes="q~U[1,4], chi~U[0,1], isotropic, omega 0.005 -> 0.05, tol 1e-8"),
    "batching_4M": Workload(
        "batching_4M", 1 << 22, ("uniform", 1.0, 10.0), ("uniform", 0.0, 1.0),
        ("loguniform", 0.002, 0.01), 0.05, 1e-8, BASE_SEED + 2,
        notes="q~U[1,10], chi~U[0,1], omega0~logU[0.002,0.01] -> 0.05, tol 1e-8"),
    "q1to4_1M_fp32split": Workload(
        "q1to4_1M_fp32split", 1 << 20, ("uniform", 1.0, 4.0), ("uniform", 0.0, 1.0),
        ("fixed", 0.005), 0.05, 1e-8, BASE_SEED + 1, precision="fp32split",
        notes="the q1to4_1M population (same seed) in the FP32-split mode"),
    "adjoint_64k": Workload(
        "adjoint_64k", 65536, ("uniform", 1.0, 4.0), ("uniform", 0.5, 1.0),
        ("fixed", 0.01), 0.05, 1e-8, BASE_SEED + 4,
        notes="q~U[1,4], chi~U[0.5,1], omega 0.01 -> 0.05, tol 1e-8"),
    # The paper's own science setting (Sec. V A) and its timing setting (Sec. IV).
    "paper_equal_mass": Workload(
        "paper_equal_mass", 4096, ("fixed", 1.0), ("fixed", 1.0, 1.0),
        ("fixed", 0.00395), 0.05, 5e-7, BASE_SEED + 10,
        notes="m_i=0.5, chi_i=1, omega 0.00395 -> 0.05, tol 5e-7 (Sec. V A)"),
    "paper_timing": Workload(
        "paper_timing", 4096, ("fixed", 1.0), ("fixed", 1.0, 1.0),
        ("fixed", 0.004), 0.1, 5e-7, BASE_SEED + 11,
        notes="m_i=0.5, chi_i=1, omega 0.004 -> 0.1, tol 5e-7: the timing run of Sec. IV "
              "(one test inspiral, replicated)"),
}


def marsaglia_sphere(rng: np.random.Generator, n: int) -> np.ndarray:
    """n points uniform on the unit sphere by Marsaglia's (1972) method.

    Draw (u1, u2) uniform on (-1, 1)^2 and keep the pairs with
    s = u1^2 + u2^2 < 1, in draw order; the point is
    (2 u1 sqrt(1-s), 2 u2 sqrt(1-s), 1 - 2 s).  Returns [3, n] float64.
    """
    out = np.empty((3, n), dtype=np.float64)
    filled = 0
    while filled < n:
        need = n - filled
        block = max(64, int(need * 1.3) + 16)
        u = rng.uniform(-1.0, 1.0, size=(block, 2))
        s = u[:, 0] ** 2 + u[:, 1] ** 2
        keep = u[s < 1.0][:need]
        sk = s[s < 1.0][:need]
        k = keep.shape[0]
        r = 2.0 * np.sqrt(1.0 - sk)
        out[0, filled:filled + k] = keep[:, 0] * r
        out[1, filled:filled + k] = keep[:, 1] * r
        out[2, filled:filled + k] = 1.0 - 2.0 * sk
        filled += k
    return out


def generate(w: Workload | str, n: int | None = None) -> dict:
    """Draw the population of workload `w` (optionally only its first n).

    The draw is always made at the workload's full size (or at n, if larger)
    and then cut, so the first n inspirals are the same for every n up to the
    workload's size; a larger n is a different draw.
    """
    if isinstance(w, str):
        w = WORKLOADS[w]
    total = w.n if n is None else max(int(n), 0)
    draw_n = max(total, w.n)
    rng = np.random.Generator(np.random.PCG64(w.seed))

    if w.q[0] == "fixed":
        q = np.full(draw_n, float(w.q[1]))
    elif w.q[0] == "uniform":
        q = rng.uniform(w.q[1], w.q[2], size=draw_n)
    else:
        raise ValueError(w.q)

    if w.chi[0] == "fixed":
        chi1 = np.full(draw_n, float(w.chi[1]))
        chi2 = np.full(draw_n, float(w.chi[2]))
    elif w.chi[0] == "uniform":
        chi1 = rng.uniform(w.chi[1], w.chi[2], size=draw_n)
        chi2 = rng.uniform(w.chi[1], w.chi[2], size=draw_n)
    else:
        raise ValueError(w.chi)

    s1 = marsaglia_sphere(rng, draw_n)
    s2 = marsaglia_sphere(rng, draw_n)

    if w.omega0[0] == "fixed":
        omega0 = np.full(draw_n, float(w.omega0[1]))
    elif w.omega0[0] == "loguniform":
        lo, hi = np.log(w.omega0[1]), np.log(w.omega0[2])
        omega0 = np.exp(rng.uniform(lo, hi, size=draw_n))
    else:
        raise ValueError(w.omega0)

    m1 = q / (1.0 + q)
    m2 = 1.0 / (1.0 + q)
    S = np.empty((6, draw_n))
    S[0:3] = chi1 * m1 ** 2 * s1
    S[3:6] = chi2 * m2 ** 2 * s2
    L = np.zeros((3, total))
    L[2] = 1.0
    return {
        "m": np.ascontiguousarray(np.stack([m1, m2])[:, :total]),
        "S": np.ascontiguousarray(S[:, :total]),
        "L": L,
        "omega0": np.ascontiguousarray(omega0[:total]),
        "chi": np.ascontiguousarray(np.stack([chi1, chi2])[:, :total]),
        "omega_f": float(w.omega_f),
        "tol": float(w.tol),
        "n": total,
        "workload": w.name,
    }


def replicate(single: dict, n: int) -> dict:
    """n copies of inspiral 0 of a population (lock-step case)."""
    out = dict(single)
    for k in ("m", "S", "L", "chi"):
        out[k] = np.ascontiguousarray(np.repeat(single[k][:, :1], n, axis=1))
    out["omega0"] = np.full(n, float(single["omega0"][0]))
    out["n"] = n
    return out


def subset(pop: dict, idx: np.ndarray) -> dict:
    """The inspirals at indices idx, as a new SoA population."""
    out = dict(pop)
    for k in ("m", "S", "L", "chi"):
        out[k] = np.ascontiguousarray(pop[k][:, idx])
    out["omega0"] = np.ascontiguousarray(pop["omega0"][idx])
    out["n"] = int(len(idx))
    return out
