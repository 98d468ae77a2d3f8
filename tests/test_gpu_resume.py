"""Resuming SBCI1 after converged roots (opts nconv0 / xc0 / ec0) through the
C ABI, against the oracle.  Between roots the solver carries only the
converged pairs {x_c, E_c} (Algorithm 1, Eqs. S4-S5 deflate against them),
so a resumed solve must take the same steps as the oracle continued from
those pairs and the same start vector."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import hamiltonian as H  # noqa: E402
from oracle import sbci as OSB  # noqa: E402
from oracle import sigma as OS  # noqa: E402
from workloads import make_integrals, start_noise  # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx(n, na, nb, rank, seed):
    import paper_2603_06101_amd as sb
    I = make_integrals(n, rank, seed)
    return sb.Context(n, na, nb, I.h1, I.eri), I


def _eigenpairs(n, na, nb, I, E, X, tol_res=3e-5):
    S = OS.sigma(n, na, nb, I.h1, I.eri, X)
    for a in range(len(E)):
        assert abs(np.linalg.norm(X[a]) - 1) < 1e-10
        assert np.linalg.norm(S[a] - E[a] * X[a]) < tol_res
    assert np.abs(X @ X.T - np.eye(len(E))).max() < 1e-8


def test_resumed_steps_match_the_oracle():
    """Root 0 solved, then roots 1 and 2 resumed from a noise start x0: every
    step (energy, b, c, |x|, restart reason) equals the oracle continued from
    the same converged pair and start."""
    n, na, nb = 7, 4, 3
    ctx, I = _ctx(n, na, nb, 14, 0)
    op = OS.Operator(n, na, nb, I.h1, I.eri)
    r0 = ctx.solve(1, tol=1e-10)
    assert r0.status == 0
    xc = r0.vectors.cpu().numpy()
    ec = np.array(r0.energies)
    x0 = np.zeros(ctx.ndet)
    x0[5] = 1.0
    x0 += 1e-2 * start_noise(n, 14, 1, ctx.ndet)
    X0 = op(x0)
    ref = OSB.sbci1(op, op.diag(), 3,
                    prev=([xc[0] / np.linalg.norm(xc[0])], [ec[0]], x0, X0, float(x0 @ X0 / (x0 @ x0))))
    ctx.begin(3, tol=1e-10, x0=x0, xc=xc, ec=ec)
    steps = []
    done = False
    while not done:
        info, done = ctx.step()
        steps.append(info)
    res = ctx.finish()
    assert res.status == 0
    assert len(steps) == len(ref.steps)
    for g, o in zip(steps, ref.steps):
        assert (g["root"], g["segment"], g["t"]) == (o.root, o.segment, o.t)
        assert abs(g["E"] - o.E) < 1e-10
        assert abs(g["b"] - o.b) < 1e-7 * max(1, abs(o.b))
        assert abs(g["c"] - o.c) < 1e-7 * max(1, abs(o.c))
        assert abs(g["xnorm"] - o.xnorm) < 1e-9
        assert g["reason"] == (o.reason or "")
    assert steps[0]["root"] == 1
    assert res.energies[0] == ec[0]
    assert np.abs(res.energies - ref.energies).max() < 1e-10
    V = res.vectors.cpu().numpy()
    assert np.abs(V[0] - xc[0]).max() < 1e-14
    assert res.report["nroots_converged"] == 3
    _eigenpairs(n, na, nb, I, res.energies, V)
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_resume_from_the_start_block_reaches_the_direct_roots(prec):
    """Root 0 given without its energy (the solver takes its Rayleigh
    quotient), root 1 onward from the Section S1.1 start block: the lowest
    three eigenvalues, as the uninterrupted solve finds them."""
    n, na, nb = 8, 5, 3
    ctx, I = _ctx(n, na, nb, 16, 2)
    w = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, I.h1, I.eri))
    d = ctx.solve(3, tol=1e-10, opts=dict(precision=prec))
    assert d.status == 0
    r1 = ctx.solve(1, tol=1e-10)
    r = ctx.solve(3, tol=1e-10, opts=dict(precision=prec), xc=r1.vectors)
    assert r.status == 0
    assert np.abs(np.asarray(r.energies) - w[:3]).max() < 1e-8
    assert np.abs(np.asarray(r.energies) - np.asarray(d.energies)).max() < 1e-8
    # the Rayleigh quotient of a converged vector: within the residual squared
    assert abs(r.energies[0] - r1.energies[0]) < 1e-9
    if prec != "f64":
        assert r.report["nsigma_low"] > 0
    _eigenpairs(n, na, nb, I, r.energies, r.vectors.cpu().numpy())
    ctx.close()


def test_given_roots_are_orthonormalised_in_order():
    """Two given roots, scaled and mixed: Gram-Schmidt in the given order
    recovers the eigenvectors, the given energies are kept, and the third
    root is the next eigenvalue."""
    n, na, nb = 7, 2, 4
    ctx, I = _ctx(n, na, nb, 14, 4)
    w = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, I.h1, I.eri))
    r2 = ctx.solve(2, tol=1e-10)
    assert r2.status == 0
    V = r2.vectors.cpu().numpy()
    mixed = np.stack([3.0 * V[0], V[1] + 0.5 * V[0]])
    r = ctx.solve(3, tol=1e-10, xc=mixed, ec=r2.energies)
    assert r.status == 0
    assert list(r.energies[:2]) == list(r2.energies)
    G = r.vectors.cpu().numpy()
    assert np.abs(G[0] - V[0]).max() < 1e-14
    assert np.abs(G[1] - V[1]).max() < 1e-9
    assert np.abs(np.asarray(r.energies) - w[:3]).max() < 1e-8
    _eigenpairs(n, na, nb, I, r.energies, G)
    ctx.close()


def test_bad_resumes_are_refused():
    import paper_2603_06101_amd as sb
    ctx, _ = _ctx(6, 3, 2, 12, 0)
    r1 = ctx.solve(1, tol=1e-10)
    v = r1.vectors.cpu().numpy()
    with pytest.raises(sb.SbciError, match="nconv0"):
        ctx.solve(1, xc=v)                                 # nothing left to solve
    with pytest.raises(sb.SbciError, match="dependent"):
        ctx.solve(3, xc=np.stack([v[0], -2.0 * v[0]]))
    with pytest.raises(sb.SbciError, match="zero"):
        ctx.solve(2, xc=np.zeros_like(v))
    with pytest.raises(sb.SbciError, match="not finite"):
        ctx.solve(2, xc=v, ec=[np.nan])
    o = sb.default_opts()
    o.nconv0 = 1                                           # no vectors given
    with pytest.raises(sb.SbciError, match="xc0"):
        ctx.solve(2, opts=o)
    keep = np.ascontiguousarray(v)
    o.xc0 = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    with pytest.raises(sb.SbciError, match="resume"):
        ctx.davidson(2, opts=o)
    with pytest.raises(sb.SbciError, match="resume"):
        ctx.solve2(2, opts=o)
    # the context still solves after the refusals
    r = ctx.solve(2, tol=1e-10, xc=v)
    assert r.status == 0 and r.report["nroots_converged"] == 2
    ctx.close()


def test_checkpoint_between_steps_and_continue():
    """A 3-root solve stopped a few steps into root 1: the converged pair
    (sbci_finish mid-solve, SBCI_ENOCONV) and the iterate (sbci_iterate) are
    the whole state, and a new context resumed from them reaches the roots of
    the uninterrupted solve.  The stopped solve itself also steps on after
    its finish call to the same roots."""
    import paper_2603_06101_amd as sb
    n, na, nb = 7, 4, 3
    ctx, I = _ctx(n, na, nb, 14, 0)
    w = np.linalg.eigvalsh(H.dense_h_slater_condon(n, na, nb, I.h1, I.eri))
    full = ctx.solve(3, tol=1e-10)
    assert full.status == 0
    with pytest.raises(sb.SbciError, match="converged"):
        ctx.iterate()                      # every root of that solve converged
    ctx.begin(3, tol=1e-10)
    done = False
    while not done:
        info, done = ctx.step()
        if info["root"] == 1 and info["t"] >= 2:
            break
    assert not done
    part = ctx.finish()
    assert part.status == sb.SBCI_ENOCONV and part.report["nroots_converged"] == 1
    xc = part.vectors[:1].cpu().numpy()
    ec = np.array(part.energies[:1])
    x = ctx.iterate().cpu().numpy()
    assert np.isfinite(x).all() and np.linalg.norm(x) > 0
    ctx2, _ = _ctx(n, na, nb, 14, 0)
    r = ctx2.solve(3, tol=1e-10, x0=x, xc=xc, ec=ec)
    assert r.status == 0
    assert np.abs(np.asarray(r.energies) - np.asarray(full.energies)).max() < 1e-8
    assert np.abs(np.asarray(r.energies) - w[:3]).max() < 1e-8
    _eigenpairs(n, na, nb, I, r.energies, r.vectors.cpu().numpy())
    ctx2.close()
    while not done:
        _, done = ctx.step()
    rest = ctx.finish()
    assert rest.status == 0
    assert np.abs(np.asarray(rest.energies) - np.asarray(full.energies)).max() < 1e-8
    ctx.close()


def test_iterate_is_refused_without_a_step_level_solve():
    import paper_2603_06101_amd as sb
    ctx, _ = _ctx(6, 3, 2, 12, 0)
    with pytest.raises(sb.SbciError):
        ctx.iterate()                      # nothing begun
    ctx.begin(2, tol=1e-10)
    ctx.step()
    assert np.isfinite(ctx.iterate().cpu().numpy()).all()
    ctx.davidson(2, tol=1e-10)             # ends the step-level solve
    with pytest.raises(sb.SbciError):
        ctx.iterate()
    ctx.solve2(2, tol=1e-10)
    with pytest.raises(sb.SbciError):
        ctx.iterate()
    ctx.close()
