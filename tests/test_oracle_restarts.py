"""Pins for the restart decisions of the oracle solvers (CPU only).

SBCI1 restarts a segment on Eq. S62a, S62b or S62c, or after max_cycle = 20
steps (Section S1.5); SBCI2 on Eq. S130a, S130b or S130c, or after
max_cycle = 10 steps (Section S2.5).  Three kinds of pins:

* hand-built states that make exactly one condition true (and its
  neighbours false), each side of every threshold, on the decision
  functions themselves;
* a closed form: on a two-level H with a constant diagonal, the first step
  lands on the exact ground state with |x_1| = 1/cos(theta), where theta is
  the angle between x_0 and the ground state, so S62b must fire exactly
  when 1/cos(theta) > x_th2;
* every recorded step of whole solves re-decided from its own recorded
  fields with the paper's conditions written out here, including
  trajectories that reach S62c / S130c and max_cycle.
"""
import math

import numpy as np
import pytest

from oracle import sbci
from oracle import sbci2
from oracle import sigma as S
from workloads import make_integrals

O1 = sbci.Options()
O2 = sbci2.Options2()


# --- the paper's thresholds (Sections S1.5, S2.5) ---------------------------

def test_thresholds_are_the_papers():
    assert (O1.b_th, O1.eps1, O1.x_th1, O1.x_th2, O1.r1, O1.max_cycle) == (1e-2, 1e-7, 0.1, 1.2, 1.0, 20)
    assert (O2.b_th, O2.eps1, O2.x_th1, O2.x_th2, O2.r1, O2.max_cycle2) == (1e-2, 1e-7, 0.1, 1.2, 1.0, 10)


# --- hand-built states, SBCI1 (Eqs. S62a-c, max_cycle) ----------------------
# A quiet state: excited root, b and dE large, |x| = 1, small residual, t = 3.
QUIET = dict(alpha=1, t=3, b=0.5, dE=1e-3, xn=1.0, dz=1e-2)


def _r1(**kw):
    a = dict(QUIET)
    a.update(kw)
    return sbci.restart_reason(a["alpha"], a["t"], a["b"], a["dE"], a["xn"], a["dz"], O1)


def test_quiet_state_does_not_restart():
    assert _r1() == ""


@pytest.mark.parametrize("xn,want", [(1.3, "S62b"), (1.2, ""), (1.2000001, "S62b"), (0.05, "S62b"),
                                     (0.1, ""), (0.0999999, "S62b"), (0.1000001, ""), (1.1999999, "")])
def test_s62b_norm_window(xn, want):
    # |x_{t+1}| outside [x_th1, x_th2] = [0.1, 1.2], strict on both ends
    assert _r1(xn=xn) == want


@pytest.mark.parametrize("t,dz,want", [(0, 2.0, ""), (1, 2.0, "S62c"), (5, 1.0, ""), (5, 1.0000001, "S62c"),
                                       (0, 50.0, "")])
def test_s62c_needs_a_large_residual_after_the_first_step(t, dz, want):
    assert _r1(t=t, dz=dz) == want


@pytest.mark.parametrize("alpha,b,dE,want", [
    (1, 5e-3, 5e-8, "S62a"),      # both small on an excited root
    (0, 5e-3, 5e-8, ""),          # the ground state never restarts on S62a
    (1, 2e-2, 5e-8, ""),          # b above b_th
    (1, 5e-3, 2e-7, ""),          # energy not settled
    (1, -5e-3, 5e-8, "S62a"),     # |b| is tested
    (1, -2e-2, 5e-8, ""),
    (2, 1e-2, 5e-8, ""),          # strict: |b| = b_th does not fire
    (2, 9.99e-3, 1e-7, ""),       # strict: dE = eps1 does not fire
])
def test_s62a_excited_roots_only(alpha, b, dE, want):
    assert _r1(alpha=alpha, b=b, dE=dE) == want


@pytest.mark.parametrize("t,want", [(18, ""), (19, "max_cycle"), (0, ""), (20, "")])
def test_max_cycle_after_twenty_steps(t, want):
    # t counts steps inside the segment from 0: step t = 19 is the 20th
    assert _r1(t=t) == want


def test_s62_order_when_several_hold():
    # the paper lists S62a, S62b, S62c; the recorded reason is the first true one
    assert _r1(b=1e-3, dE=1e-9, xn=5.0, dz=9.0) == "S62a"
    assert _r1(xn=5.0, dz=9.0) == "S62b"
    assert _r1(dz=9.0, t=19) == "S62c"


# --- hand-built states, SBCI2 (Eqs. S130a-c, max_cycle) ---------------------

def _r2b(b00=0.5, b11=0.5, dE=1e-3, k0=1.0, k1=1.0):
    return sbci2.restart_reason_before_update(np.array([[b00, 0.3], [0.2, b11]]), dE,
                                              np.array([k0, k1]), O2)


def test_s130a_either_diagonal_of_B():
    assert _r2b() == ""
    assert _r2b(b00=5e-3, dE=5e-8) == "S130a"
    assert _r2b(b11=-5e-3, dE=5e-8) == "S130a"
    assert _r2b(b00=5e-3, dE=2e-7) == ""          # energy of state alpha not settled
    assert _r2b(b00=1e-2, b11=1e-2, dE=5e-8) == ""  # strict
    # the off-diagonal entries of B play no part
    assert sbci2.restart_reason_before_update(np.array([[0.5, 1e-9], [1e-9, 0.5]]), 1e-9,
                                              np.array([1.0, 1.0]), O2) == ""


@pytest.mark.parametrize("k0,k1,want", [(1.3, 1.0, "S130b"), (1.0, 1.3, "S130b"), (0.05, 1.0, "S130b"),
                                        (1.0, 0.05, "S130b"), (1.2, 0.1, ""), (1.19, 0.11, "")])
def test_s130b_either_norm(k0, k1, want):
    assert _r2b(k0=k0, k1=k1) == want


@pytest.mark.parametrize("t,dz,want", [(0, 2.0, ""), (1, 2.0, "S130c"), (4, 1.0, ""), (8, 0.5, ""),
                                       (9, 0.5, "max_cycle"), (9, 3.0, "S130c")])
def test_s130c_and_max_cycle_ten(t, dz, want):
    assert sbci2.restart_reason_after_update(t, dz, O2) == want


# --- closed form: |x_1| = 1/cos(theta) on a two-level H ---------------------

def _two_level(theta, d=-1.0, e=0.5):
    A = np.array([[d, e], [e, d]])               # ground state (1, -1)/sqrt 2 at d - e
    u0 = np.array([1.0, -1.0]) / math.sqrt(2)
    u1 = np.array([1.0, 1.0]) / math.sqrt(2)
    x0 = math.cos(theta) * u0 + math.sin(theta) * u1

    def op(v):
        return np.atleast_2d(v) @ A.T if np.ndim(v) > 1 else A @ v
    return op, np.diag(A).copy(), x0, d - e


@pytest.mark.parametrize("deg", [10.0, 25.0, 33.0, 34.0, 40.0, 44.0])
def test_s62b_closed_form_on_a_two_level_h(deg):
    """With a constant diagonal the preconditioned residual is orthogonal to
    x_0, span{x_0, z} is the whole space, the lowest Ritz vector is the
    ground state u_0 and x_1 = k u_0 with k = 1/(u_0 . x_0) = 1/cos(theta)
    (Eqs. S17, S23).  S62b fires iff 1/cos(theta) > 1.2 (theta > 33.56 deg)."""
    th = math.radians(deg)
    op, D, x0, E0 = _two_level(th)
    r = sbci.sbci1(op, D, 1, opts=sbci.Options(max_steps=1), x0=x0)
    s = r.steps[0]
    assert s.t == 0 and s.root == 0
    assert abs(s.xnorm - 1 / math.cos(th)) < 1e-12
    assert abs(s.E - E0) < 1e-13
    assert s.dz < 1e-12                      # x_1 is the exact eigenvector
    assert abs(s.dE - 2 * 0.5 * math.sin(th) ** 2) < 1e-12   # E_0 = d - e cos 2 theta
    assert s.reason == ("S62b" if 1 / math.cos(th) > 1.2 else "")


# --- every recorded step re-decided from its own fields ---------------------

def _paper_s62(s, o):
    """Eqs. S62a-c and max_cycle, written out from Section S1.5."""
    if s.root > 0 and abs(s.b) < o.b_th and s.dE < o.eps1:
        return "S62a"
    if s.xnorm < o.x_th1 or s.xnorm > o.x_th2:
        return "S62b"
    if s.dz > o.r1 and s.t > 0:
        return "S62c"
    if s.t + 1 == o.max_cycle:
        return "max_cycle"
    return ""


def _check_sbci1_trajectory(r, o):
    seen = set()
    for s in r.steps:
        if s.reason in ("rank", "coef"):
            continue
        conv = s.dE < o.eps0 and s.dz < o.r0                       # Eq. S61
        if conv:
            assert s.reason == "converged", s
        else:
            assert s.reason == _paper_s62(s, o), s
        seen.add(s.reason)
    # segments never run past max_cycle steps
    assert all(s.t < o.max_cycle for s in r.steps)
    # after a restart the next step starts a new segment at t = 0
    for a, b in zip(r.steps, r.steps[1:]):
        if a.reason and a.reason != "converged" and b.root == a.root:
            assert b.t == 0 and b.segment == a.segment + 1, (a, b)
        elif not a.reason and b.root == a.root:
            assert b.t == a.t + 1 and b.segment == a.segment, (a, b)
    return seen


def _prob(n, na, nb, K, seed):
    I = make_integrals(n, K, seed)
    return S.Operator(n, na, nb, I.h1, I.eri)


def test_sbci1_trajectories_follow_section_S1_5():
    seen = set()
    for (n, na, nb, nr, seed, mc) in [(6, 3, 3, 4, 0, 20), (7, 3, 3, 3, 1, 20), (8, 4, 4, 3, 0, 5),
                                      (6, 3, 3, 4, 2, 3)]:
        op = _prob(n, na, nb, 2 * n, seed)
        o = sbci.Options(max_cycle=mc)
        r = sbci.sbci1(op, op.diag(), nr, o)
        assert r.converged
        seen |= _check_sbci1_trajectory(r, o)
    assert {"S62a", "S62b", "max_cycle", "converged", ""} <= seen


def _scaled_random(n=40, seed=0):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    A = 50 * (M + M.T) + np.diag(np.arange(n) * 30.0)

    def op(v):
        return np.atleast_2d(v) @ A if np.ndim(v) > 1 else A @ v
    return op, np.diag(A).copy(), A


def test_sbci1_s62c_fires_only_after_the_first_step():
    """A strongly coupled H (residual norms >> r1): steps at t = 0 with
    |z'| > r1 must not restart on S62c, steps at t > 0 must."""
    op, D, A = _scaled_random()
    o = sbci.Options()
    r = sbci.sbci1(op, D, 3, o)
    assert r.converged
    seen = _check_sbci1_trajectory(r, o)
    assert "S62c" in seen
    big0 = [s for s in r.steps if s.t == 0 and s.dz > o.r1 and s.reason not in ("rank", "coef")]
    assert big0 and all(s.reason != "S62c" for s in big0)
    w = np.linalg.eigvalsh(A)
    for E in r.energies:
        assert np.min(np.abs(w - E)) < 1e-8 * np.abs(w).max()


def _paper_s130(s, o, early):
    if early:
        if (abs(s.b00) < o.b_th or abs(s.b11) < o.b_th) and s.dE < o.eps1:
            return "S130a"
        if s.kn0 < o.x_th1 or s.kn1 < o.x_th1 or s.kn0 > o.x_th2 or s.kn1 > o.x_th2:
            return "S130b"
        return ""
    if s.dz > o.r1 and s.t > 0:
        return "S130c"
    if s.t + 1 == o.max_cycle2:
        return "max_cycle"
    return ""


def _check_sbci2_trajectory(r, o):
    seen = set()
    for s in r.steps:
        if s.reason == "coef":
            continue
        early = _paper_s130(s, o, True)
        conv = s.dE < o.eps0 and s.dz < o.r0                       # Eq. S127
        if conv:
            assert s.reason == "converged", s
        elif early:
            assert s.reason == early, s
        else:
            assert s.reason == _paper_s130(s, o, False), s
        seen.add(s.reason)
    assert all(s.t < o.max_cycle2 for s in r.steps)
    return seen


def test_sbci2_trajectories_follow_section_S2_5():
    seen = set()
    for (n, na, nb, nr, seed, mc) in [(6, 3, 3, 4, 0, 10), (7, 3, 3, 3, 1, 10), (8, 4, 4, 3, 0, 5),
                                      (6, 3, 3, 4, 2, 3)]:
        op = _prob(n, na, nb, 2 * n, seed)
        o = sbci2.Options2(max_cycle2=mc)
        r = sbci2.sbci2(op, op.diag(), nr, o)
        assert r.converged
        seen |= _check_sbci2_trajectory(r, o)
    assert {"S130a", "S130b", "max_cycle", "converged", ""} <= seen


def test_sbci2_s130c_fires_only_after_the_first_step():
    op, D, A = _scaled_random(seed=1)
    o = sbci2.Options2()
    r = sbci2.sbci2(op, D, 3, o)
    seen = _check_sbci2_trajectory(r, o)
    assert "S130c" in seen
    big0 = [s for s in r.steps if s.t == 0 and s.dz > o.r1 and s.reason not in ("coef",)]
    assert big0 and all(s.reason != "S130c" for s in big0)
