"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and assembles integral arrays from
them; it contains none of the eigensolver or sigma arithmetic, so both the
CPU oracle and the HIP path can consume the same inputs without sharing
method code.

Integral recipe (the paper's molecular instances need an integral engine,
which is absent; these seeded integrals stand in for them with the same
orbital counts and the same 8-fold symmetric structure):

  1. rng = numpy.random.default_rng(seed)        (PCG64)
  2. h[p, p] = -1.0 + 0.25 * p                    (0-based p)
  3. u ~ N(0,1), N(N-1)/2 draws in triu_indices(N, 1) order:
         h[p, q] = h[q, p] = 0.05 * u
  4. for k in 1..K: v ~ N(0,1), N(N+1)/2 draws in triu_indices(N) order:
         L_k[p, q] = L_k[q, p] = 0.1 * v * exp(-|p - q| / 4)
  5. (pq|rs) = sum_k L_k[p, q] * L_k[r, s]        (PSD as an N^2 x N^2 matrix)

Every step gives the same bits on every host: the normal draws are PCG64's,
exp(-d/4) is correctly rounded from decimal arithmetic, and the sum in step 5
runs over k in order, one elementwise product and add at a time (no BLAS).

Point-group symmetric variant (``make_sym_integrals``): orbital p carries the
D2h-like irrep label orbsym[p] (``orbital_irreps``: p mod 8); after the same
draws, h[p, q] is kept only where orbsym[p] == orbsym[q], and L_k only on the
orbital pairs whose irrep product orbsym[p] ^ orbsym[q] equals k mod 8.  Then
(pq|rs) vanishes unless the four labels XOR to zero (totally symmetric
integrals) and stays PSD.
"""
from __future__ import annotations

import decimal
import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Integrals",
    "make_integrals",
    "start_noise",
    "sigma_inputs",
    "batch_instances",
    "orbital_irreps",
    "make_sym_integrals",
    "CONFIGS",
]


@dataclass(frozen=True)
class Integrals:
    norb: int
    rank: int
    seed: int
    h1: np.ndarray   # [norb, norb] float64, symmetric
    eri: np.ndarray  # [norb, norb, norb, norb] float64, chemists' (pq|rs)

    def digest(self) -> str:
        m = hashlib.sha256()
        m.update(np.ascontiguousarray(self.h1).tobytes())
        m.update(np.ascontiguousarray(self.eri).tobytes())
        return m.hexdigest()


def _draw(norb: int, rank: int, rng: np.random.Generator, orbsym=None):
    n = norb
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = -1.0 + 0.25 * np.arange(n)
    iu = np.triu_indices(n, 1)
    u = rng.standard_normal(len(iu[0]))
    h[iu] = 0.05 * u
    h[(iu[1], iu[0])] = 0.05 * u
    it = np.triu_indices(n)
    damp = _damping(n)[np.abs(it[0] - it[1])]
    L = np.zeros((rank, n, n))
    for k in range(rank):
        v = rng.standard_normal(len(it[0]))
        L[k][it] = 0.1 * v * damp
        L[k][(it[1], it[0])] = 0.1 * v * damp
    if orbsym is not None:
        g = np.asarray(orbsym, dtype=np.int64)
        pair = g[:, None] ^ g[None, :]
        h = np.where(pair == 0, h, 0.0)
        for k in range(rank):
            L[k] = np.where(pair == (k % 8), L[k], 0.0)
    # sum over k in order, one elementwise product and add per k: the same
    # bits on every host (a BLAS product would sum in a host-dependent order)
    Lm = L.reshape(rank, n * n)
    eri = np.zeros((n * n, n * n))
    for k in range(rank):
        eri += np.multiply.outer(Lm[k], Lm[k])
    return h, eri.reshape(n, n, n, n)


def _damping(n: int) -> np.ndarray:
    """exp(-d / 4) for d = 0 .. n-1, correctly rounded (40-digit decimal
    arithmetic, then the nearest double), so the value does not depend on
    the host's exp implementation."""
    ctx = decimal.Context(prec=40)
    return np.array([float(ctx.exp(decimal.Decimal(-d) / 4)) for d in range(n)])


def make_integrals(norb: int, rank: int, seed: int) -> Integrals:
    """Seeded integrals G(norb, rank, seed) following the recipe above."""
    rng = np.random.default_rng(seed)
    h, eri = _draw(norb, rank, rng)
    return Integrals(norb, rank, seed, h, eri)


def orbital_irreps(norb: int) -> np.ndarray:
    """D2h-like irrep labels 0..7 of the orbitals (orbital p carries p mod 8)."""
    return np.arange(norb, dtype=np.int64) % 8


def make_sym_integrals(norb: int, rank: int, seed: int, orbsym=None) -> Integrals:
    """Seeded totally symmetric integrals (the symmetric variant of the recipe)."""
    if orbsym is None:
        orbsym = orbital_irreps(norb)
    rng = np.random.default_rng(seed)
    h, eri = _draw(norb, rank, rng, orbsym)
    return Integrals(norb, rank, seed, h, eri)


def start_noise(norb: int, rank: int, seed: int, ndet: int) -> np.ndarray:
    """Gaussian noise for the 'lowest determinant + 1e-3 noise' start vector.

    Drawn from the same generator as the integrals, after the integral draws,
    so the start vector is a pure function of (norb, rank, seed).
    Returns xi (unscaled, N(0,1)); the caller forms e_0 + 1e-3 * xi.
    """
    rng = np.random.default_rng(seed)
    _draw(norb, rank, rng)
    return rng.standard_normal(ndet)


def sigma_inputs(seed: int, nvec: int, ndet: int, dtype=np.float64) -> np.ndarray:
    """Dense normalised random vectors [nvec, ndet] for sigma throughput and parity."""
    rng = np.random.default_rng(seed + 7)
    c = rng.standard_normal((nvec, ndet))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    return c.astype(dtype)


def batch_instances(count: int = 512, master_seed: int = 2603):
    """Instance list for the batching workload: (norb, nelec_per_spin, nroots, seed).

    norb uniform in 6..10, n_alpha = n_beta = floor(norb / 2), 1..3 roots,
    integrals G(norb, 2 * norb, seed=i).
    """
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(count):
        norb = int(rng.integers(6, 11))
        nroots = int(rng.integers(1, 4))
        out.append((norb, norb // 2, nroots, i))
    return out


# The five workloads: (name, norb, n_alpha, n_beta, eri rank, seed, nroots)
CONFIGS = {
    "cas6": dict(norb=6, na=3, nb=3, rank=12, seed=0, nroots=1),
    "cas10": dict(norb=10, na=5, nb=5, rank=20, seed=0, nroots=3),
    "cas14": dict(norb=14, na=7, nb=7, rank=28, seed=0, nroots=5),
    "cas16": dict(norb=16, na=8, nb=8, rank=32, seed=0, nroots=1),
    # few electrons in many orbitals: the shape of the paper's CAS(6e,45o)
    # instance (201,356,100 determinants), where most orbital pairs connect a
    # string to nothing
    "dilute45": dict(norb=45, na=3, nb=3, rank=90, seed=0, nroots=1),
    # the shape of the paper's CAS(8e,29o) instance (564,110,001 determinants):
    # one row of sigma (23,751 beta strings) exceeds LDS
    "dilute29": dict(norb=29, na=4, nb=4, rank=58, seed=0, nroots=1),
    # point-group blocked: CAS(14e,14o) with orbital irreps p mod 8 and
    # totally symmetric integrals, lowest states of irrep 0
    # (1,472,928 of the 11,778,624 determinants)
    "cas14_sym": dict(norb=14, na=7, nb=7, rank=28, seed=0, nroots=5, irrep=0),
    # CAS(16e,16o) blocked the same way (20,708,900 determinants), ground state
    "cas16_sym": dict(norb=16, na=8, nb=8, rank=32, seed=0, nroots=1, irrep=0),
}
