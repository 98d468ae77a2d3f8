"""Determinant-basis Hamiltonian (oracle): two independent dense builders.

The paper's problem is the lowest eigenpairs of the electronic Hamiltonian
represented in Slater determinants (Results, "SBCI1 algorithm").  With real
one-electron integrals h_pq and chemists' two-electron integrals (pq|rs):

    H = sum_pq h_pq sum_u a+_(p,u) a_(q,u)
        + 1/2 sum_pqrs (pq|rs) sum_(u,v) a+_(p,u) a+_(r,v) a_(s,v) a_(q,u)

(u, v run over the two spin labels.)

Determinant |Ia, Ib> = prod_{p in Ia, ascending} a+_{p alpha}
                      prod_{q in Ib, ascending} a+_{q beta} |vac>,
i.e. spin orbitals are ordered alpha block first; index = Ia * Nb + Ib.

Builder 1 (``dense_h_bruteforce``) applies every operator term to every
determinant.  Builder 2 (``dense_h_slater_condon``) uses the Slater-Condon
rules with signs from occupied-orbital counts.  They share only the string
enumeration.  ``hdiag`` is the closed-form diagonal and ``spin_square`` the
textbook <S^2> = Sz^2 + (Na + Nb)/2 - sum_pq <E^a_pq E^b_qp>.
"""
from __future__ import annotations

import numpy as np

from . import strings as _st


def _det_list(norb, na, nb):
    sa = [int(m) for m in _st.strings(norb, na)]
    sb = [int(m) for m in _st.strings(norb, nb)]
    dets = [(a | (b << norb)) for a in sa for b in sb]
    return dets


# ---------------------------------------------------------------- builder 1
def _ann(mask, k):
    if not (mask >> k) & 1:
        return None, 0
    return mask & ~(1 << k), -1 if bin(mask & ((1 << k) - 1)).count("1") & 1 else 1


def _cre(mask, k):
    if (mask >> k) & 1:
        return None, 0
    return mask | (1 << k), -1 if bin(mask & ((1 << k) - 1)).count("1") & 1 else 1


def dense_h_bruteforce(norb, na, nb, h1, eri):
    """H by applying each term of the second-quantised operator (spin orbitals)."""
    dets = _det_list(norb, na, nb)
    index = {d: i for i, d in enumerate(dets)}
    n = len(dets)
    H = np.zeros((n, n))
    nso = 2 * norb
    sp = lambda k: k // norb          # spin of spin-orbital k
    orb = lambda k: k % norb          # spatial orbital of spin-orbital k
    for col, d in enumerate(dets):
        occ = [k for k in range(nso) if (d >> k) & 1]
        # one-body: a+_P a_Q, same spin
        for Q in occ:
            d1, s1 = _ann(d, Q)
            for P in range(nso):
                if sp(P) != sp(Q):
                    continue
                d2, s2 = _cre(d1, P)
                if d2 is None:
                    continue
                H[index[d2], col] += h1[orb(P), orb(Q)] * s1 * s2
        # two-body: 1/2 (pq|rs) a+_P a+_R a_S a_Q, spin(P)=spin(Q), spin(R)=spin(S)
        for Q in occ:
            d1, s1 = _ann(d, Q)
            for S in occ:
                d2, s2 = _ann(d1, S)
                if d2 is None:
                    continue
                for R in range(nso):
                    if sp(R) != sp(S):
                        continue
                    d3, s3 = _cre(d2, R)
                    if d3 is None:
                        continue
                    for P in range(nso):
                        if sp(P) != sp(Q):
                            continue
                        d4, s4 = _cre(d3, P)
                        if d4 is None:
                            continue
                        H[index[d4], col] += 0.5 * eri[orb(P), orb(Q), orb(R), orb(S)] \
                            * s1 * s2 * s3 * s4
    return H


# ---------------------------------------------------------------- builder 2
def _between(mask, a, b):
    lo, hi = (a, b) if a < b else (b, a)
    return bin(mask & (((1 << hi) - 1) ^ ((1 << (lo + 1)) - 1))).count("1")


def dense_h_slater_condon(norb, na, nb, h1, eri):
    """H from the Slater-Condon rules on spin-orbital determinants."""
    dets = _det_list(norb, na, nb)
    index = {d: i for i, d in enumerate(dets)}
    n = len(dets)
    H = np.zeros((n, n))
    nso = 2 * norb
    sp = lambda k: k // norb
    orb = lambda k: k % norb

    def g(P, Q, R, S):  # physicists' <PQ|RS> = (pr|qs) with spin deltas
        if sp(P) != sp(R) or sp(Q) != sp(S):
            return 0.0
        return eri[orb(P), orb(R), orb(Q), orb(S)]

    def gas(P, Q, R, S):  # antisymmetrised <PQ||RS>
        return g(P, Q, R, S) - g(P, Q, S, R)

    def hso(P, Q):
        return h1[orb(P), orb(Q)] if sp(P) == sp(Q) else 0.0

    for col, d in enumerate(dets):
        occ = [k for k in range(nso) if (d >> k) & 1]
        vir = [k for k in range(nso) if not (d >> k) & 1]
        # diagonal
        e = sum(hso(P, P) for P in occ)
        e += 0.5 * sum(gas(P, Q, P, Q) for P in occ for Q in occ)
        H[col, col] += e
        # singles Q -> P
        for Q in occ:
            for P in vir:
                if sp(P) != sp(Q):
                    continue
                nd = (d & ~(1 << Q)) | (1 << P)
                sgn = -1 if _between(d, P, Q) & 1 else 1
                v = hso(P, Q) + sum(gas(P, R, Q, R) for R in occ if R != Q)
                H[index[nd], col] += sgn * v
        # doubles (Q1<Q2) -> (P1<P2)
        for i1, Q1 in enumerate(occ):
            for Q2 in occ[i1 + 1:]:
                for j1, P1 in enumerate(vir):
                    for P2 in vir[j1 + 1:]:
                        if sp(P1) + sp(P2) != sp(Q1) + sp(Q2):
                            continue
                        v = gas(P1, P2, Q1, Q2)
                        if v == 0.0:
                            continue
                        # sign: move Q2 -> P2 first, then Q1 -> P1
                        d1 = (d & ~(1 << Q2)) | (1 << P2)
                        s1 = -1 if _between(d, P2, Q2) & 1 else 1
                        d2 = (d1 & ~(1 << Q1)) | (1 << P1)
                        s2 = -1 if _between(d1, P1, Q1) & 1 else 1
                        H[index[d2], col] += s1 * s2 * v
    return H


# ---------------------------------------------------------------- diagonal
def hdiag(norb, na, nb, h1, eri):
    """Closed-form diagonal D[Ia, Ib] (used by the preconditioner (D - E0)^-1, Eq. 7 context)."""
    sa = _st.strings(norb, na)
    sb = _st.strings(norb, nb)
    J = np.einsum("ppqq->pq", eri)
    K = np.einsum("pqqp->pq", eri)

    def occ_mat(ss):
        return np.array([[(int(m) >> p) & 1 for p in range(norb)] for m in ss], dtype=float)

    oa, ob = occ_mat(sa), occ_mat(sb)
    hd = np.diag(h1)
    ea = oa @ hd + 0.5 * np.einsum("ip,pq,iq->i", oa, J - K, oa)
    eb = ob @ hd + 0.5 * np.einsum("ip,pq,iq->i", ob, J - K, ob)
    cross = oa @ J @ ob.T
    return (ea[:, None] + eb[None, :] + cross).reshape(-1)


# ---------------------------------------------------------------- spin
def spin_square(norb, na, nb, c):
    """<S^2> of a vector c [Na * Nb] (textbook second-quantised expression)."""
    c = np.asarray(c, dtype=float).reshape(-1)
    sa = [int(m) for m in _st.strings(norb, na)]
    sb = [int(m) for m in _st.strings(norb, nb)]
    ia = {m: i for i, m in enumerate(sa)}
    ib = {m: i for i, m in enumerate(sb)}
    C = c.reshape(len(sa), len(sb))
    W = np.zeros_like(C)
    # w = sum_pq E^a_pq E^b_qp c
    for p in range(norb):
        for q in range(norb):
            # E^b_qp on beta strings
            bmap = []
            for j, m in enumerate(sb):
                nm, s = _st.apply_epq(m, q, p)
                if nm is not None:
                    bmap.append((j, ib[nm], s))
            if not bmap:
                continue
            amap = []
            for j, m in enumerate(sa):
                nm, s = _st.apply_epq(m, p, q)
                if nm is not None:
                    amap.append((j, ia[nm], s))
            if not amap:
                continue
            ja = np.array([a[0] for a in amap]); ka = np.array([a[1] for a in amap])
            sa_ = np.array([a[2] for a in amap], dtype=float)
            jb = np.array([b[0] for b in bmap]); kb = np.array([b[1] for b in bmap])
            sb_ = np.array([b[2] for b in bmap], dtype=float)
            W[np.ix_(ka, kb)] += sa_[:, None] * sb_[None, :] * C[np.ix_(ja, jb)]
    sz = 0.5 * (na - nb)
    nrm = float(c @ c)
    return sz * sz + 0.5 * (na + nb) - float(C.reshape(-1) @ W.reshape(-1)) / nrm
