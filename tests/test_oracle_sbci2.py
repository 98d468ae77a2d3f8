"""Pins of the SBCI2 oracle (Algorithm 2, Sections S2.1-S2.5) against
independent mathematics: a QR-based Rayleigh-Ritz for the pair update and the
dense Slater-Condon spectrum for whole solves."""
import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import sbci2 as S2
from oracle import sigma as OS
from workloads import make_integrals


def _ritz_qr(basis, Hfull):
    """Rayleigh-Ritz in span(basis) by QR (independent of canonical orthogonalisation)."""
    Q, _ = np.linalg.qr(basis.T)
    w, V = np.linalg.eigh(Q.T @ Hfull @ Q)
    return w, (Q @ V).T


def _parallel(u, v):
    return abs(u @ v) / (np.linalg.norm(u) * np.linalg.norm(v))


@pytest.mark.parametrize("seed", range(6))
def test_pair_update_gives_the_two_lowest_ritz_vectors(seed):
    """Eqs. S103-S125: with A, B, C from the two lowest Ritz vectors, the updated
    x^a, x^a+1 are parallel to them (Eq. S110) and carry their Ritz values."""
    rng = np.random.default_rng(seed)
    n = 40
    G = rng.standard_normal((n, n))
    Hf = 0.5 * (G + G.T) + np.diag(np.linspace(-3, 3, n))
    x = rng.standard_normal((2, n))
    y = 0.3 * rng.standard_normal((2, n))
    z = 0.1 * rng.standard_normal((2, n))
    basis = np.vstack([x, y, z])
    S = basis @ basis.T
    Hm = basis @ Hf @ basis.T
    w, Vp = S2.canonical_ritz(S, Hm, 1e-14)
    cf = S2.coefficients_next(Vp, 1e-14)
    A, B, C = cf["A"], cf["B"], cf["C"]
    y1 = y - C @ z + A @ x
    x1 = x + B @ y1
    wq, Rq = _ritz_qr(basis, Hf)
    assert np.allclose(w[:2], wq[:2], atol=1e-10)
    # V' is orthonormal in the overlap metric, so |x_{t+1}| = |k| (what the
    # S130b test before the update relies on)
    assert np.allclose(Vp.T @ S @ Vp, np.eye(Vp.shape[1]), atol=1e-10)
    for i in range(2):
        assert abs(np.linalg.norm(x1[i]) - abs(cf["k"][i])) < 1e-8
    for i in range(2):
        assert _parallel(x1[i], Rq[i]) > 1 - 1e-10
        assert abs(x1[i] @ Hf @ x1[i] / (x1[i] @ x1[i]) - wq[i]) < 1e-10
        assert abs(abs(cf["k"][i]) * np.linalg.norm(basis.T @ Vp[:, i]) - np.linalg.norm(x1[i])) < 1e-8


@pytest.mark.parametrize("seed", range(6))
def test_first_pair_step_gives_the_two_lowest_ritz_vectors(seed):
    """Eqs. S83-S97 (t = 0, y = 0, B = I): x_1 = x_0 + A x_0 - C z_0 is parallel
    to the two lowest Ritz vectors of span{x^a, x^a+1, z^a, z^a+1}."""
    rng = np.random.default_rng(100 + seed)
    n = 30
    G = rng.standard_normal((n, n))
    Hf = 0.5 * (G + G.T)
    x = rng.standard_normal((2, n))
    x /= np.linalg.norm(x, axis=1)[:, None]
    z = 0.05 * rng.standard_normal((2, n))
    basis = np.vstack([x, z])
    w, Vp = S2.canonical_ritz(basis @ basis.T, basis @ Hf @ basis.T, 1e-14)
    cf = S2.coefficients_first(Vp, 1e-14)
    x1 = x + cf["A"] @ x - cf["C"] @ z
    wq, Rq = _ritz_qr(basis, Hf)
    for i in range(2):
        assert _parallel(x1[i], Rq[i]) > 1 - 1e-10
        assert abs(w[i] - wq[i]) < 1e-10


def test_canonical_orthogonalisation_drops_dependent_vectors():
    """Overlap eigenvalues <= 1e-14 are dropped (Section S2.3): a duplicated
    vector leaves the Ritz values of the independent span unchanged."""
    rng = np.random.default_rng(7)
    n = 20
    G = rng.standard_normal((n, n))
    Hf = 0.5 * (G + G.T)
    v = rng.standard_normal((3, n))
    basis = np.vstack([v, v[1]])          # rank 3 in a 4-vector basis
    w, Vp = S2.canonical_ritz(basis @ basis.T, basis @ Hf @ basis.T, 1e-14)
    assert len(w) == 3
    wq, _ = _ritz_qr(v, Hf)
    assert np.allclose(w, wq, atol=1e-10)


@pytest.mark.parametrize("n,na,nb,nroots,seed", [(6, 3, 3, 3, 0), (6, 2, 2, 4, 2), (7, 3, 4, 3, 3),
                                                 (8, 4, 4, 3, 5), (5, 2, 3, 2, 1)])
def test_sbci2_roots_are_eigenpairs(n, na, nb, nroots, seed):
    I = make_integrals(n, 2 * n, seed)
    op = OS.Operator(n, na, nb, I.h1, I.eri)
    r = S2.sbci2(op, op.diag(), nroots)
    assert r.converged
    Hd = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    w = np.linalg.eigvalsh(Hd)
    X = r.vectors
    assert np.abs(X @ X.T - np.eye(nroots)).max() < 1e-8
    for a, E in enumerate(r.energies):
        assert np.min(np.abs(w - E)) < 1e-8
        assert np.linalg.norm(Hd @ X[a] - E * X[a]) < 1e-4
    # from the two-vector start the pairs reach the lowest states in order
    assert abs(r.energies[0] - w[0]) < 1e-8


def test_sbci2_single_root_is_sbci1():
    from oracle import sbci as S1
    I = make_integrals(6, 12, 0)
    op = OS.Operator(6, 3, 3, I.h1, I.eri)
    r2 = S2.sbci2(op, op.diag(), 1)
    r1 = S1.sbci1(op, op.diag(), 1)
    assert abs(r2.energies[0] - r1.energies[0]) < 1e-12


@pytest.mark.parametrize("n,na,nb,nroots,seed", [(6, 2, 2, 4, 2), (7, 3, 4, 3, 3), (8, 4, 4, 5, 1)])
def test_sbci2_energies_are_rayleigh_quotients(n, na, nb, nroots, seed):
    """Each returned energy is the Rayleigh quotient of its returned vector when
    the projections of Eq. S78 / Section S2.2 use the carried images H x_c.
    With E_c x_c as printed, the residual of the accepted x_c stays in X and
    the later energies drift from the Rayleigh quotients (first order in it)."""
    I = make_integrals(n, 2 * n, seed)
    op = OS.Operator(n, na, nb, I.h1, I.eri)
    gaps = []
    for images in (True, False):
        r = S2.sbci2(op, op.diag(), nroots, S2.Options2(s78_images=images), record=False)
        X = r.vectors
        rq = np.einsum("ij,ij->i", X, np.atleast_2d(op(X)))
        gaps.append(np.abs(r.energies - rq).max())
    assert gaps[0] < 1e-12
    assert gaps[1] > 1e-9
