"""Pins for the oracle's strings, addressing and excitation tables (CPU only)."""
import os
from math import comb

import numpy as np
import pytest

from oracle import strings as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ndet_section_S3_1.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, n, a, b, nd = line.split()
        rows.append((name, int(n), int(a), int(b), int(nd)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[0])
def test_ndet_matches_paper_table(row):
    # Section S3.1 prints N_det for every instance; the string count is C(N, m).
    name, n, a, b, nd = row
    assert comb(n, a) * comb(n, b) == nd


@pytest.mark.parametrize("n,m", [(1, 0), (1, 1), (4, 2), (6, 3), (8, 3), (10, 5), (12, 4)])
def test_strings_enumeration_and_address(n, m):
    s = st.strings(n, m)
    assert len(s) == comb(n, m)
    assert np.all(np.diff(s.astype(np.int64)) > 0) if len(s) > 1 else True
    for i, mask in enumerate(s):
        assert bin(int(mask)).count("1") == m
        assert st.address(int(mask)) == i


def _between(mask, p, q):
    lo, hi = min(p, q), max(p, q)
    return sum((mask >> r) & 1 for r in range(lo + 1, hi))


@pytest.mark.parametrize("n,m", [(4, 2), (6, 3), (7, 2), (5, 5), (5, 0), (8, 4)])
def test_excitation_table_properties(n, m):
    J, P, Q, S = st.excitation_table(n, m)
    strs = st.strings(n, m)
    ns = len(strs)
    assert J.shape == (ns, m * (n - m + 1))
    entries = {}
    for i in range(ns):
        mask = int(strs[i])
        # diagonal entries first: E_pp |I> = |I>, so sum_p E_pp |I> = m |I>
        for e in range(m):
            assert P[i, e] == Q[i, e] and J[i, e] == i and S[i, e] == 1
        for e in range(J.shape[1]):
            p, q, j, s = int(P[i, e]), int(Q[i, e]), int(J[i, e]), int(S[i, e])
            # sign from the count of occupied orbitals strictly between p and q
            assert s == (-1) ** _between(mask, p, q)
            # target string = I - q + p
            assert int(strs[j]) == (mask & ~(1 << q)) | (1 << p)
            entries[(i, p, q)] = (j, s)
    # hermiticity: (p,q,J,s) of I <=> (q,p,I,s) of J
    for (i, p, q), (j, s) in entries.items():
        assert entries[(j, q, p)] == (i, s)


def test_table_order_is_occ_then_virt():
    J, P, Q, S = st.excitation_table(6, 3)
    strs = st.strings(6, 3)
    mask = int(strs[7])
    occ = [p for p in range(6) if (mask >> p) & 1]
    vir = [p for p in range(6) if not (mask >> p) & 1]
    want = [(o, o) for o in occ] + [(p, q) for q in occ for p in vir]
    assert list(zip(P[7].tolist(), Q[7].tolist())) == want
