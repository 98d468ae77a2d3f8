"""Occupation strings, lexical addressing and single-excitation tables (oracle).

Definitions (the paper works in a Slater-determinant basis, Results "SBCI1
algorithm"; the determinant count of Section S3.1 is C(norb, n_alpha) *
C(norb, n_beta)):

* A string is an m-subset of orbitals {0..N-1}, stored as an integer bit
  mask (bit p set <=> orbital p occupied).  Strings are ordered by ascending
  mask value.
* E_pq = a+_p a_q acting on a string.  For q occupied and (p empty or p == q)
  E_pq |I> = sign |I - q + p>, sign = (-1)^(number of occupied orbitals
  strictly between p and q); otherwise 0.  The sign is obtained here by
  literally applying a_q and then a+_p to an ordered product of creators.
* Table order per string: the m diagonal entries (p == q, ascending), then
  q over occupied orbitals ascending, p over empty orbitals ascending.

Everything here is brute force on Python integers; it is only run on small
orbital counts by the tests, and at up to 16 orbitals for table parity.
"""
from __future__ import annotations

from itertools import combinations
from math import comb

import numpy as np


def strings(norb: int, nelec: int) -> np.ndarray:
    """All nelec-subsets of norb orbitals as uint64 masks, ascending."""
    masks = [sum(1 << p for p in occ) for occ in combinations(range(norb), nelec)]
    return np.array(sorted(masks), dtype=np.uint64)


def address(mask: int) -> int:
    """Rank of a string among same-size strings in ascending mask order.

    Combinatorial number system: occupied o_1 < ... < o_m (0-based) have
    rank sum_k C(o_k, k).  Pinned by tests against ``strings`` (rank == index).
    """
    occ = [p for p in range(64) if (mask >> p) & 1]
    return sum(comb(o, k + 1) for k, o in enumerate(occ))


def _annihilate(mask: int, q: int):
    if not (mask >> q) & 1:
        return None, 0
    below = bin(mask & ((1 << q) - 1)).count("1")
    return mask & ~(1 << q), (-1) ** below


def _create(mask: int, p: int):
    if (mask >> p) & 1:
        return None, 0
    below = bin(mask & ((1 << p) - 1)).count("1")
    return mask | (1 << p), (-1) ** below


def apply_epq(mask: int, p: int, q: int):
    """E_pq |mask> by explicit operator application: (new_mask, sign) or (None, 0)."""
    m1, s1 = _annihilate(mask, q)
    if m1 is None:
        return None, 0
    m2, s2 = _create(m1, p)
    if m2 is None:
        return None, 0
    return m2, s1 * s2


def excitation_table(norb: int, nelec: int):
    """Single-excitation table of every string.

    Returns (J, p, q, sign) arrays of shape [nstr, s] with
    s = nelec * (norb - nelec + 1):  E_pq |I> = sign |J>.
    """
    strs = strings(norb, nelec)
    index = {int(m): i for i, m in enumerate(strs)}
    nstr = len(strs)
    s = nelec * (norb - nelec + 1)
    J = np.zeros((nstr, s), dtype=np.int32)
    P = np.zeros((nstr, s), dtype=np.uint8)
    Q = np.zeros((nstr, s), dtype=np.uint8)
    S = np.zeros((nstr, s), dtype=np.int8)
    for i, m in enumerate(strs):
        m = int(m)
        occ = [p for p in range(norb) if (m >> p) & 1]
        vir = [p for p in range(norb) if not (m >> p) & 1]
        e = 0
        for o in occ:
            nm, sg = apply_epq(m, o, o)
            J[i, e], P[i, e], Q[i, e], S[i, e] = index[nm], o, o, sg
            e += 1
        for q in occ:
            for p in vir:
                nm, sg = apply_epq(m, p, q)
                J[i, e], P[i, e], Q[i, e], S[i, e] = index[nm], p, q, sg
                e += 1
    return J, P, Q, S


def packed_table(norb: int, nelec: int) -> np.ndarray:
    """The table as 8-byte records: int32 J, uint8 p, uint8 q, int8 sign, uint8 0."""
    J, P, Q, S = excitation_table(norb, nelec)
    rec = np.zeros(J.shape, dtype=np.dtype([("J", "<i4"), ("p", "u1"), ("q", "u1"),
                                            ("sign", "i1"), ("pad", "u1")]))
    rec["J"], rec["p"], rec["q"], rec["sign"] = J, P, Q, S
    return rec
