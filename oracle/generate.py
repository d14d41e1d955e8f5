"""CPU oracle of the on-device population generator: the counter-based
Philox4x64-10 generator (Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC11) and the draw of masses, spins and
initial frequencies from its streams (the initial data of Sec. II and V).

TEST INFRASTRUCTURE: only the tests use it.  numpy uint64 arithmetic,
written from the published definition; it shares nothing with the GPU
library.

Stream layout (the same on the GPU): inspiral i draws from the blocks
Philox((i, k, 0, 0), key), k = 0, 1, ...; block 0 gives the uniforms of q,
chi_1, chi_2, omega0; blocks 1..32 the Marsaglia attempts of S_hat_1 (two
attempts per block), blocks 33..64 those of S_hat_2.  A uniform is
(x >> 11) * 2^-53 in [0, 1).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
MASK32 = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)
MAX_ATTEMPTS = 64


def mulhilo(a: np.ndarray, b: np.uint64):
    """The 128-bit product a*b as (hi, lo) 64-bit words."""
    a = np.asarray(a, dtype=np.uint64)
    al, ah = a & MASK32, a >> S32
    bl, bh = b & MASK32, b >> S32
    p0, p1, p2, p3 = al * bl, al * bh, ah * bl, ah * bh
    mid = (p0 >> S32) + (p1 & MASK32) + (p2 & MASK32)
    hi = p3 + (p1 >> S32) + (p2 >> S32) + (mid >> S32)
    return hi, a * b


def philox4x64(ctr, key) -> np.ndarray:
    """Philox4x64-10 of counters ctr [4, ...] under key (k0, k1): ten rounds of
    (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
    lo(M0 x0)), the key advanced by the Weyl constants between rounds."""
    with np.errstate(over="ignore"):
        x = [np.asarray(c, dtype=np.uint64).copy() for c in ctr]
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        for r in range(10):
            if r:
                k0, k1 = k0 + W0, k1 + W1
            hi0, lo0 = mulhilo(x[0], M0)
            hi1, lo1 = mulhilo(x[2], M1)
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return np.stack(x)


def uniform(words: np.ndarray) -> np.ndarray:
    """(x >> 11) 2^-53: a double in [0, 1)."""
    return (np.asarray(words, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def _block(i: np.ndarray, k: int, key) -> np.ndarray:
    z = np.zeros_like(i)
    return philox4x64([i, np.full_like(i, k), z, z], key)


def _sphere(i: np.ndarray, first_block: int, key) -> np.ndarray:
    """Marsaglia (1972): the first attempt (u1, u2) in (-1, 1)^2 with
    s = u1^2 + u2^2 < 1 gives (2 u1 sqrt(1-s), 2 u2 sqrt(1-s), 1 - 2s);
    z = (0, 0, 1) if none of the MAX_ATTEMPTS is accepted."""
    n = i.size
    out = np.zeros((3, n))
    out[2] = 1.0
    done = np.zeros(n, bool)
    for a in range(MAX_ATTEMPTS):
        w = _block(i, first_block + a // 2, key)
        u1 = 2.0 * uniform(w[2 * (a % 2)]) - 1.0
        u2 = 2.0 * uniform(w[2 * (a % 2) + 1]) - 1.0
        s = u1 * u1 + u2 * u2
        take = ~done & (s < 1.0)
        r = 2.0 * np.sqrt(1.0 - s[take])
        out[0, take] = u1[take] * r
        out[1, take] = u2[take] * r
        out[2, take] = 1.0 - 2.0 * s[take]
        done |= take
        if done.all():
            break
    return out


def _param(spec, u):
    """('fixed', v) -> v;  ('uniform', lo, hi) -> lo + (hi - lo) u."""
    if spec[0] == "fixed":
        return np.full(u.shape, float(spec[1]))
    lo, hi = float(spec[1]), float(spec[2])
    return lo + (hi - lo) * u


def population(n: int, seed: int, q, chi, omega0, first: int = 0) -> dict:
    """Inspirals first .. first + n - 1 of the stream with key (seed, 0):
    M = 1, m1 = q/(1 + q), m2 = 1/(1 + q), S_i = chi_i m_i^2 S_hat_i,
    L_hat = z, omega0; q, chi_i and omega0 fixed or uniform (spec tuples as
    above; chi as ('fixed', c1, c2) or ('uniform', lo, hi))."""
    key = (np.uint64(seed), np.uint64(0))
    i = np.arange(first, first + n, dtype=np.uint64)
    w = _block(i, 0, key)
    q = _param(q, uniform(w[0]))
    if chi[0] == "fixed":
        c1 = np.full(n, float(chi[1]))
        c2 = np.full(n, float(chi[2]))
    else:
        c1 = _param(chi, uniform(w[1]))
        c2 = _param(chi, uniform(w[2]))
    w0 = _param(omega0, uniform(w[3]))
    m1 = q / (1.0 + q)
    m2 = 1.0 / (1.0 + q)
    s1 = _sphere(i, 1, key)
    s2 = _sphere(i, 1 + MAX_ATTEMPTS // 2, key)
    a1 = c1 * (m1 * m1)
    a2 = c2 * (m2 * m2)
    S = np.concatenate([a1 * s1, a2 * s2])
    L = np.zeros((3, n))
    L[2] = 1.0
    return {"m": np.stack([m1, m2]), "S": S, "L": L, "omega0": w0}
