"""Pins for the oracle Hamiltonian, diagonal, sigma and <S^2> (CPU only)."""
from math import comb

import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import sigma as S
from workloads import make_integrals


def _ints(n, seed=3):
    I = make_integrals(n, 2 * n, seed)
    return I.h1, I.eri


@pytest.mark.parametrize("n,na,nb", [(3, 1, 1), (4, 2, 2), (4, 2, 1), (4, 0, 2), (4, 4, 1),
                                     (5, 2, 3), (6, 3, 3)])
def test_two_dense_builders_agree(n, na, nb):
    h, g = _ints(n)
    Hb = H.dense_h_bruteforce(n, na, nb, h, g)
    Hs = H.dense_h_slater_condon(n, na, nb, h, g)
    assert Hb.shape == (comb(n, na) * comb(n, nb),) * 2
    assert np.abs(Hb - Hs).max() < 1e-13
    assert np.abs(Hs - Hs.T).max() < 1e-14
    assert np.abs(np.diag(Hs) - H.hdiag(n, na, nb, h, g)).max() < 1e-13


@pytest.mark.parametrize("n,na,nb", [(4, 2, 2), (5, 2, 3), (6, 3, 3), (6, 2, 4), (6, 6, 0), (7, 3, 3)])
def test_c_sigma_equals_dense(n, na, nb):
    h, g = _ints(n, seed=5)
    Hs = H.dense_h_slater_condon(n, na, nb, h, g)
    rng = np.random.default_rng(1)
    c = rng.standard_normal((2, Hs.shape[0]))
    sg = S.sigma(n, na, nb, h, g, c)
    assert np.abs(sg - c @ Hs).max() < 1e-12
    d = S.hdiag(n, na, nb, h, g, Hs.shape[0])
    assert np.abs(d - np.diag(Hs)).max() < 1e-13
    rows = np.unique(np.array([0, min(3, Hs.shape[0] - 1), Hs.shape[0] - 1]))
    assert np.abs(S.sigma_rows(n, na, nb, h, g, c[0], rows) - (Hs @ c[0])[rows]).max() < 1e-12


def test_sigma_invariants_cas8():
    n, na, nb = 8, 4, 4
    h, g = _ints(n, seed=7)
    nd = comb(8, 4) ** 2
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal((2, nd))
    a, b = 0.7, -1.3
    su, sv = S.sigma(n, na, nb, h, g, np.stack([u, v]))
    # linearity
    assert np.abs(S.sigma(n, na, nb, h, g, a * u + b * v) - (a * su + b * sv)).max() < 1e-12
    # symmetry u^T H v = v^T H u
    assert abs(u @ sv - v @ su) < 1e-11 * np.sqrt(nd)
    # transpose symmetry for n_alpha = n_beta
    ns = comb(8, 4)
    U = u.reshape(ns, ns)
    st = S.sigma(n, na, nb, h, g, U.T.reshape(-1)).reshape(ns, ns)
    assert np.abs(st - su.reshape(ns, ns).T).max() < 1e-12


def test_closed_form_no_two_electron():
    # eri = 0: eigenvalues are sums of orbital energies; ground = lowest na + lowest nb
    n, na, nb = 5, 2, 2
    h, _ = _ints(n)
    g = np.zeros((n,) * 4)
    eps = np.linalg.eigvalsh(h)
    Hs = H.dense_h_slater_condon(n, na, nb, h, g)
    e0 = np.linalg.eigvalsh(Hs)[0]
    assert abs(e0 - (eps[:na].sum() + eps[:nb].sum())) < 1e-12


def test_closed_form_one_electron_each_spin():
    # na = nb = 1: H[(p,q),(r,s)] = h_pr d_qs + d_pr h_qs + (pr|qs)
    n = 4
    h, g = _ints(n)
    Hs = H.dense_h_slater_condon(n, 1, 1, h, g)
    want = np.einsum("pr,qs->pqrs", h, np.eye(n)) + np.einsum("pr,qs->pqrs", np.eye(n), h) \
        + np.einsum("prqs->pqrs", g)
    assert np.abs(Hs - want.reshape(n * n, n * n)).max() < 1e-13


def test_closed_form_single_spin():
    n = 5
    h, g = _ints(n)
    Hs = H.dense_h_slater_condon(n, 1, 0, h, g)
    assert np.abs(np.linalg.eigvalsh(Hs) - np.linalg.eigvalsh(h)).max() < 1e-13


def test_closed_form_fully_occupied():
    n = 4
    h, g = _ints(n)
    Hs = H.dense_h_slater_condon(n, n, n, h, g)
    want = 2 * np.trace(h) + sum(2 * g[p, p, q, q] - g[p, q, q, p] for p in range(n) for q in range(n))
    assert Hs.shape == (1, 1) and abs(Hs[0, 0] - want) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.5, 1.0), (1.0, 0.0)])
def test_two_site_hubbard(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2,) * 4)
    g[0, 0, 0, 0] = g[1, 1, 1, 1] = U
    Hs = H.dense_h_bruteforce(2, 1, 1, h, g)
    e0 = np.linalg.eigvalsh(Hs)[0]
    assert abs(e0 - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-13


def test_orbital_rotation_invariance():
    n, na, nb = 5, 2, 2
    h, g = _ints(n, seed=11)
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    h2 = Q.T @ h @ Q
    g2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", g, Q, Q, Q, Q)
    e1 = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, h, g))
    e2 = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, h2, g2))
    assert np.abs(e1 - e2).max() < 1e-10


def test_spin_square_of_eigenvectors():
    n, na, nb = 5, 2, 2
    h, g = _ints(n, seed=2)
    w, v = np.linalg.eigh(H.dense_h_slater_condon(n, na, nb, h, g))
    for i in range(6):
        if min(abs(w[i] - w[j]) for j in range(len(w)) if j != i) < 1e-8:
            continue
        s2 = H.spin_square(n, na, nb, v[:, i])
        S_ = round((np.sqrt(1 + 4 * s2) - 1) / 2)
        assert abs(s2 - S_ * (S_ + 1)) < 1e-8
    # a single closed-shell determinant is a singlet; an open-shell one mixes
    e0 = np.zeros(len(w)); e0[0] = 1.0
    assert abs(H.spin_square(n, na, nb, e0)) < 1e-14
    # high-spin single determinant (na=2, nb=0) has S(S+1) = 2
    e1 = np.zeros(comb(n, 2)); e1[0] = 1.0
    assert abs(H.spin_square(n, 2, 0, e1) - 2.0) < 1e-14
