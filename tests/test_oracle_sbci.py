"""Pins for the oracle SBCI1 step algebra and solvers (CPU only)."""
from math import comb

import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import sbci
from oracle import sigma as S
from workloads import make_integrals, start_noise


def _rayleigh_ritz(A, vecs):
    """Independent Rayleigh-Ritz: QR basis, projected matrix, eigh."""
    Q, _ = np.linalg.qr(np.array(vecs).T)
    w, u = np.linalg.eigh(Q.T @ A @ Q)
    return w, Q @ u


@pytest.mark.parametrize("seed", range(6))
def test_ritz_next_matches_independent_rayleigh_ritz(seed):
    rng = np.random.default_rng(seed)
    n = 30
    M = rng.standard_normal((n, n))
    A = 0.5 * (M + M.T)
    x, y, z = rng.standard_normal((3, n))
    x *= 0.9
    X, Y, Z = A @ x, A @ y, A @ z
    N = dict(xx=x @ x, xy=x @ y, xz=x @ z, yy=y @ y, yz=y @ z, zz=z @ z)
    Hm = dict(xx=x @ X, xy=x @ Y, xz=x @ Z, yy=y @ Y, yz=y @ Z, zz=z @ Z)
    r = sbci.ritz_next(N, Hm, 1e-14)
    w, V = _rayleigh_ritz(A, [x, y, z])
    assert np.abs(r["E"] - w).max() < 1e-12
    b, c, k = r["b"], r["c"], r["k"]
    xn = x + b * y - b * c * z              # Eq. S47
    assert abs(np.linalg.norm(xn) - abs(k)) < 1e-12 * abs(k)   # Eq. S62b: |k| = |x_{t+1}|
    cosang = abs(xn @ V[:, 0]) / np.linalg.norm(xn)
    assert cosang > 1 - 1e-12
    # second Ritz vector from the coefficients on (x, y, z) (Section S1.4)
    a = r["coef"][1]
    v2 = a[0] * x + a[1] * y + a[2] * z
    assert abs(np.linalg.norm(v2) - 1) < 1e-12
    assert abs(abs(v2 @ V[:, 1]) - 1) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_ritz_first_matches_independent_rayleigh_ritz(seed):
    rng = np.random.default_rng(100 + seed)
    n = 20
    M = rng.standard_normal((n, n))
    A = 0.5 * (M + M.T)
    x, z = rng.standard_normal((2, n))
    x /= np.linalg.norm(x)                  # the first step assumes |x0| = 1
    X, Z = A @ x, A @ z
    r = sbci.ritz_first(x @ x, x @ z, z @ z, x @ X, x @ Z, z @ Z, 1e-14)
    w, V = _rayleigh_ritz(A, [x, z])
    assert np.abs(r["E"] - w).max() < 1e-12
    x1 = x - r["c"] * z                     # Eq. S18 with b0 = 1
    assert abs(np.linalg.norm(x1) - abs(r["k"])) < 1e-12 * abs(r["k"])
    assert abs(x1 @ V[:, 0]) / np.linalg.norm(x1) > 1 - 1e-12


def _problem(n, na, nb, rank, seed):
    I = make_integrals(n, rank, seed)
    op = S.Operator(n, na, nb, I.h1, I.eri)
    return I, op


def test_sbci1_cfg0_start_converges_to_an_eigenpair():
    n, na, nb, K = 6, 3, 3, 12
    I, op = _problem(n, na, nb, K, 0)
    Hs = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    w = np.linalg.eigvalsh(Hs)
    xi = start_noise(n, K, 0, op.ndet)
    x0 = np.zeros(op.ndet); x0[0] = 1.0
    r = sbci.sbci1(op, op.diag(), 1, x0=x0 + 1e-3 * xi)
    assert r.converged
    E = r.energies[0]
    assert np.min(np.abs(w - E)) < 1e-8          # an eigenvalue of H
    assert E >= w[0] - 1e-12                      # variational bound
    x = r.vectors[0]
    assert np.linalg.norm(Hs @ x - E * x) < 1e-5


@pytest.mark.parametrize("n,na,nb,nroots,seed", [(6, 3, 3, 4, 0), (6, 3, 3, 3, 2), (7, 4, 3, 3, 0),
                                                 (6, 2, 3, 2, 1)])
def test_sbci1_roots_are_eigenpairs(n, na, nb, nroots, seed):
    I, op = _problem(n, na, nb, 2 * n, seed)
    Hs = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    w = np.linalg.eigvalsh(Hs)
    r = sbci.sbci1(op, op.diag(), nroots)
    assert r.converged and len(r.energies) == nroots
    for a in range(nroots):
        E, x = r.energies[a], r.vectors[a]
        assert np.min(np.abs(w - E)) < 1e-8
        assert np.linalg.norm(Hs @ x - E * x) < 2e-5
    G = r.vectors @ r.vectors.T
    assert np.abs(G - np.eye(nroots)).max() < 1e-8
    # energies never increase within a segment (lowest Ritz value of a space containing x_t)
    prev = None
    for s in r.steps:
        if prev is not None and s.root == prev.root and s.segment == prev.segment and s.t > 0:
            assert s.E <= prev.E + 1e-12 * abs(prev.E)
        prev = s
    # restart reasons are the paper's
    assert {s.reason for s in r.steps} <= {"", "converged", "S62a", "S62b", "S62c", "max_cycle",
                                           "rank", "coef"}


def test_sbci1_excited_roots_orthogonal_and_s2():
    n, na, nb = 6, 3, 3
    I, op = _problem(n, na, nb, 12, 2)
    r = sbci.sbci1(op, op.diag(), 3)
    for a in range(3):
        s2 = H.spin_square(n, na, nb, r.vectors[a])
        S_ = round((np.sqrt(1 + 4 * s2) - 1) / 2)
        assert abs(s2 - S_ * (S_ + 1)) < 1e-6


@pytest.mark.parametrize("n,na,nb,nroots,seed", [(6, 3, 3, 4, 0), (7, 3, 3, 3, 1)])
def test_davidson_matches_eigh(n, na, nb, nroots, seed):
    I, op = _problem(n, na, nb, 2 * n, seed)
    w = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, I.h1, I.eri))
    r = sbci.davidson(op, op.diag(), nroots)
    assert r.converged
    for E in r.energies:
        assert np.min(np.abs(w - E)) < 1e-8


def test_start_vectors_section_S1_1():
    n, na, nb = 6, 3, 3
    I, op = _problem(n, na, nb, 12, 0)
    d = op.diag()
    x0, X0, E = sbci.start_vectors(op, d, 3)
    order = np.lexsort((np.arange(len(d)), d))[:3]
    assert np.allclose(np.abs(x0).sum(axis=0)[np.setdiff1d(np.arange(len(d)), order)], 0)
    Hs = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    sub = Hs[np.ix_(order, order)]
    assert np.abs(np.sort(E) - np.linalg.eigvalsh(sub)).max() < 1e-13
    assert np.abs(X0 - x0 @ Hs).max() < 1e-13


def test_stored_cas14_roots_are_the_lowest_lanczos_values():
    """The stored CAS(14,14) run (tests/golden/make_refs.py, oracle only): the
    five SBCI1 roots (Algorithm 1 with the deflated excited roots of Section
    S1.4) are the five lowest eigenvalues that an independent Lanczos solver
    (scipy eigsh on the oracle's sigma) finds, below a sixth one."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "refs.json")))["cas14"]
    assert ref["digest"] == make_integrals(14, 28, 0).digest()
    e = np.sort(np.array(ref["sbci1"]))
    lan = np.array(ref["eigsh"])
    assert len(lan) == 6 and ref["sbci1_converged"]
    assert np.abs(e - lan[:5]).max() < 1e-9
    assert lan[5] - e[-1] > 1e-3


@pytest.mark.parametrize("n,na,nb,seed", [(6, 3, 2, 0), (7, 4, 3, 1), (6, 2, 3, 2)])
def test_sbci1_continued_after_given_roots_reaches_the_next_eigenvalues(n, na, nb, seed):
    """The continuation path (prev = converged pairs and a start): with the
    exact lowest eigenpair of the dense H given as converged and a start that
    still overlaps it strongly, the projection of the root start (Eqs. S4-S5)
    and the deflated steps (Eq. S31) lead to the next two eigenvalues, with
    vectors orthogonal to the given one."""
    I, op = _problem(n, na, nb, 2 * n, seed)
    Hs = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    w, V = np.linalg.eigh(Hs)
    rng = np.random.default_rng(seed)
    x0 = V[:, 0] + 0.3 * V[:, 1] + 0.05 * rng.standard_normal(Hs.shape[0])
    X0 = op(x0)
    r = sbci.sbci1(op, op.diag(), 3, prev=([V[:, 0]], [w[0]], x0, X0, float(x0 @ X0 / (x0 @ x0))))
    assert r.converged and len(r.energies) == 3
    assert r.energies[0] == w[0]
    assert np.abs(r.energies[1:] - w[1:3]).max() < 1e-8
    for a in (1, 2):
        x = r.vectors[a]
        assert abs(x @ V[:, 0]) < 1e-8
        assert np.linalg.norm(Hs @ x - r.energies[a] * x) < 2e-5
    assert {s.root for s in r.steps} == {1, 2}
