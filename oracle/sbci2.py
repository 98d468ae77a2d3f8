"""SBCI2 reference in FP64 NumPy (oracle; test infrastructure only).

SBCI2 (Algorithm 2, Supplementary Sections S2.1-S2.5) solves the states of a
pair (alpha, alpha + 1) together and accepts state alpha when it converges;
the highest state is finished with SBCI1 (Fig. 1B).  This module follows the
paper's steps in its order and notation:

* start vectors: the n lowest diagonal determinants, H diagonalised in their
  span (Eqs. S74-S76); the partner of a later pair is the next such vector,
  orthogonalised against the converged roots and against x_0^alpha
  (Section S2.2);
* pair start: project both vectors off the converged roots and normalise
  (Eqs. S77-S80, the pair start of Algorithm 2); y = Y = 0, B = I at each
  segment start;
* each step: both preconditioned, deflated residuals (Eqs. S81 / S101) and
  their sigma images (Eqs. S82 / S102); the basis (x^a, x^a+1, z^a, z^a+1) at
  t = 0 or (x^a, x^a+1, y^a, y^a+1, z^a, z^a+1) at t >= 1 is orthonormalised
  canonically (overlap eigenvalues <= 1e-14 dropped) and H is diagonalised
  in it (Eqs. S83-S87 / S103-S107); A, B, C follow from the two lowest Ritz
  vectors (Eqs. S93 at t = 0, S112-S121 at t >= 1); y, Y, x, X are updated
  (Eqs. S94-S97 / S122-S125) and the residuals formed (Eqs. S98/S100,
  S126/S128);
* state alpha converges on Eq. S127; otherwise the pair restarts on S130a,
  S130b, S130c or after max_cycle = 10 steps (Section S2.5).

Readings of points the paper leaves open:
  residual scale 1/|x| (Algorithm 2's residual); preconditioner shift E^0 = the
  current energy of state 0 while alpha = 0, else E_c^0, |D - E^0| floored
  at 1e-8; a restart (back to the segment start) zeroes y and uses the t = 0
  step; a
  vanishing denominator of the coefficient formulas, or fewer than two kept
  basis vectors, restarts the pair from its two lowest Ritz vectors (or
  from the normalised x's); the partner's starting energy is its Rayleigh
  quotient after the projection of Section S2.2.
  Eq. S78 (and the same projection in Section S2.2) takes E_c x_c for the
  image H x_c of a converged root, which holds for an exact eigenvector
  only.  An accepted x_c still carries a residual r_c (|z'| < r0), and the
  printed form leaves r_c (x_c . x) in X for good: the Ritz energies of the
  later states then differ from the Rayleigh quotients of their vectors at
  first order in r_c (10^-8 - 10^-7 Eh at 12-14 orbitals), because the
  partner from Eq. S75 overlaps the converged roots strongly.  The image
  carried to acceptance (X of the accepted state, normalised) is H x_c up to
  rounding, so the projection uses it (s78_images = True, the default);
  s78_images = False keeps the printed E_c x_c.
  S130a and S130b need only the step's coefficients (|x_{t+1}| = |k|, since
  the updated vectors are k times S-orthonormal Ritz vectors), so they are
  tested before the update, and their restart takes the two Ritz vectors
  from the basis: identical to normalising the updated vectors in exact
  arithmetic, but free of the cancellation x_t + B y ~ 0 that the update
  suffers when |k| << 1, which otherwise leaves X inconsistent with H x.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import sbci as S1


@dataclass
class Options2(S1.Options):
    max_cycle2: int = 10    # Section S2.5
    s78_images: bool = True  # H x_c from the carried image in Eq. S78 (reading)


@dataclass
class PairStep:
    alpha: int
    segment: int
    t: int
    E: float
    E2: float
    dE: float
    dz: float
    reason: str
    # the step's B_t diagonal and |k| (= |x_{t+1}|) of both states (NaN for
    # a coefficient restart), recorded for the Section S2.5 tests
    b00: float = float("nan")
    b11: float = float("nan")
    kn0: float = float("nan")
    kn1: float = float("nan")


def canonical_ritz(Smat, Hmat, lindep):
    """Canonical orthogonalisation and Rayleigh-Ritz (Eqs. S83-S87, S103-S107).

    Smat, Hmat: overlap and H in the (non-orthogonal) basis.  Returns the
    Ritz values w (ascending) and V' = P V, the Ritz vectors' coefficients on
    the basis, or None when fewer than two basis vectors survive.
    """
    s, U = np.linalg.eigh(0.5 * (Smat + Smat.T))
    keep = s > lindep
    if keep.sum() < 2:
        return None
    P = U[:, keep] / np.sqrt(s[keep])              # P = U s^-1/2
    Hp = P.T @ (0.5 * (Hmat + Hmat.T)) @ P
    w, V = np.linalg.eigh(0.5 * (Hp + Hp.T))
    return w, P @ V


def coefficients_first(Vp, lindep):
    """Eqs. S92-S93: k, A, C of the first step (basis x^a, x^a+1, z^a, z^a+1)."""
    d0, d1 = Vp[0, 0], Vp[1, 1]
    if abs(d0) < lindep or abs(d1) < lindep:
        return None
    k0, k1 = 1.0 / d0, 1.0 / d1
    a01, a10 = Vp[1, 0] / d0, Vp[0, 1] / d1
    C = np.array([[-Vp[2, 0] / d0, -Vp[3, 0] / d0],
                  [-Vp[2, 1] / d1, -Vp[3, 1] / d1]])
    return dict(k=(k0, k1), A=np.array([[0.0, a01], [a10, 0.0]]), B=np.eye(2), C=C)


def coefficients_next(Vp, lindep):
    """Eqs. S112-S121: k, A, B, C of a later step (basis x^a, x^a+1, y^a, y^a+1, z^a, z^a+1)."""
    if abs(Vp[2, 0]) < lindep or abs(Vp[3, 1]) < lindep:
        return None
    a01 = Vp[1, 0] / Vp[2, 0]                      # S116
    a10 = Vp[0, 1] / Vp[3, 1]
    den0 = Vp[0, 0] - Vp[3, 0] * a10               # S117
    den1 = Vp[1, 1] - Vp[2, 1] * a01
    if abs(den0) < lindep or abs(den1) < lindep:
        return None
    k0, k1 = 1.0 / den0, 1.0 / den1
    B = np.array([[k0 * Vp[2, 0], k0 * Vp[3, 0]],  # S112
                  [k1 * Vp[2, 1], k1 * Vp[3, 1]]])
    M = np.array([[Vp[2, 0], Vp[3, 0]], [Vp[2, 1], Vp[3, 1]]])
    R = np.array([[Vp[4, 0], Vp[5, 0]], [Vp[4, 1], Vp[5, 1]]])
    if abs(np.linalg.det(M)) < lindep * max(1e-300, np.abs(M).max() ** 2):
        return None
    C = -np.linalg.solve(M, R)                     # S121
    return dict(k=(k0, k1), A=np.array([[0.0, a01], [a10, 0.0]]), B=B, C=C)


def restart_reason_before_update(B, dE, kn, o: Options2) -> str:
    """Section S2.5, the conditions fixed by the step's coefficients.

    B: the 2x2 B_t of the step, dE = |E_{t+1}^alpha - E_t^alpha|, kn: the two
    norms |x_{t+1}^alpha|, |x_{t+1}^alpha+1| (= |k|).  Eq. S130a: either
    diagonal entry of B below b_th while state alpha's energy has settled;
    Eq. S130b: either norm outside [x_th1, x_th2].  Strict comparisons."""
    if (abs(B[0, 0]) < o.b_th or abs(B[1, 1]) < o.b_th) and dE < o.eps1:
        return "S130a"
    if (kn[0] < o.x_th1 or kn[1] < o.x_th1 or kn[0] > o.x_th2 or kn[1] > o.x_th2):
        return "S130b"
    return ""


def restart_reason_after_update(t, dz, o: Options2) -> str:
    """Section S2.5 after the update: Eq. S130c (|z'^alpha_{t+1}| above r1,
    not on a segment's first step), then max_cycle (10) steps in the segment."""
    if dz > o.r1 and t > 0:
        return "S130c"
    if t + 1 == o.max_cycle2:
        return "max_cycle"
    return ""


@dataclass
class Result2:
    energies: np.ndarray
    vectors: np.ndarray
    nsigma: int
    steps: list = field(default_factory=list)
    converged: bool = True


def sbci2(op, diag, nroots, opts: Options2 | None = None, record=True):
    """Lowest nroots eigenpairs of H by SBCI2 (Algorithm 2, Fig. 1B).  op(v) = H v."""
    o = opts or Options2()
    diag = np.asarray(diag, dtype=np.float64)
    ndet = diag.shape[0]
    if nroots == 1 or ndet < 2:
        r = S1.sbci1(op, diag, nroots, o, record=False)
        return Result2(r.energies, r.vectors, r.nsigma, [], r.converged)
    xs, Xs, Es = S1.start_vectors(op, diag, nroots)       # Eqs. S74-S76
    nsig = nroots
    xc, Ec, Xcs = [], [], []
    steps = []
    all_conv = True

    def floor_den(E0):
        den = diag - E0
        return np.where(np.abs(den) < o.precond_floor, o.precond_floor, den)

    def images():
        # H x_c of the converged roots: carried images, or E_c x_c (Eq. S78 as printed)
        if o.s78_images:
            return np.array(Xcs)
        return np.array(Ec)[:, None] * np.array(xc)

    def deflate(w):
        if not xc:
            return w
        Xc = np.array(xc)
        return w - Xc.T @ (Xc @ w)

    # pair (0, 1): x_0^0, x_0^1 from Eq. S75
    xa, Xa = xs[0].copy(), Xs[0].copy()
    xb, Xb = xs[1].copy(), Xs[1].copy()
    for alpha in range(nroots - 1):
        # the pair start of Algorithm 2 (Eqs. S77-S80)
        xv, Xv = [xa, xb], [Xa, Xb]
        for i in range(2):
            if xc:
                Xc = np.array(xc)
                proj = Xc @ xv[i]
                xv[i] = xv[i] - Xc.T @ proj
                Xv[i] = Xv[i] - images().T @ proj
            nrm = np.linalg.norm(xv[i])
            xv[i], Xv[i] = xv[i] / nrm, Xv[i] / nrm
        x = np.array(xv)
        X = np.array(Xv)
        E = np.array([x[i] @ X[i] for i in range(2)])
        seg = 0
        nstep = 0
        conv = False
        while not conv:
            # segment start: y = Y = 0, B = I, z' = (H - E) x / |x|
            y = np.zeros((2, ndet))
            Y = np.zeros((2, ndet))
            zp = np.array([(X[i] - E[i] * x[i]) / np.linalg.norm(x[i]) for i in range(2)])
            t = 0
            while True:
                E0 = E[0] if alpha == 0 else Ec[0]
                den = floor_den(E0)
                z = np.array([deflate(zp[i] / den) for i in range(2)])   # S81 / S101
                Z = np.atleast_2d(op(z))                                  # S82 / S102
                nsig += 2
                nstep += 1
                if t == 0:
                    basis = np.vstack([x, z])
                    imgs = np.vstack([X, Z])
                else:
                    basis = np.vstack([x, y, z])
                    imgs = np.vstack([X, Y, Z])
                Smat = basis @ basis.T
                Hmat = basis @ imgs.T
                rr = canonical_ritz(Smat, Hmat, o.lindep)
                cf = None
                if rr is not None:
                    w, Vp = rr
                    cf = coefficients_first(Vp, o.lindep) if t == 0 else coefficients_next(Vp, o.lindep)
                if cf is None:
                    # restart the pair from its two lowest Ritz vectors (or from x)
                    if rr is not None:
                        v = Vp[:, :2].T @ basis
                        V = Vp[:, :2].T @ imgs
                        E = np.array(w[:2], dtype=float)
                    else:
                        v, V = x, X
                    nv = np.linalg.norm(v, axis=1)
                    x, X = v / nv[:, None], V / nv[:, None]
                    if rr is None:
                        E = np.array([x[i] @ X[i] for i in range(2)])
                    if record:
                        steps.append(PairStep(alpha, seg, t, E[0], E[1], np.nan, np.nan, "coef"))
                    seg += 1
                    break
                Enew = np.array(w[:2], dtype=float)
                A, B, C = cf["A"], cf["B"], cf["C"]
                dE = abs(Enew[0] - E[0])
                # S130a and S130b are decided by the step's coefficients: the
                # updated vectors are k times the two lowest Ritz vectors, which
                # are orthonormal in the overlap metric, so |x_{t+1}| = |k|
                kn = np.abs(np.array(cf["k"], dtype=float))
                early = restart_reason_before_update(B, dE, kn, o)
                if early:
                    # restart (Section S2.5): x_{t+1}/|x_{t+1}| are the Ritz vectors
                    # themselves; take them from the basis, since the update
                    # reaches them through cancellation when |k| << 1
                    v = Vp[:, :2].T @ basis
                    V = Vp[:, :2].T @ imgs
                    nv = np.linalg.norm(v, axis=1)
                    x, X = v / nv[:, None], V / nv[:, None]
                    dz = np.linalg.norm(X[0] - Enew[0] * x[0])
                    conv = dE < o.eps0 and dz < o.r0                              # S127
                    reason = "converged" if conv else early
                    if record:
                        steps.append(PairStep(alpha, seg, t, Enew[0], Enew[1], dE, dz, reason,
                                              B[0, 0], B[1, 1], kn[0], kn[1]))
                    E = Enew
                    if not conv:
                        seg += 1
                    break
                if t == 0:
                    # Eqs. S94-S97: y_1 = A x_0 - C z_0, x_1 = x_0 + y_1
                    y = A @ x - C @ z
                    Y = A @ X - C @ Z
                    x = x + y
                    X = X + Y
                else:
                    # Eqs. S122-S125
                    y = y - C @ z + A @ x
                    Y = Y - C @ Z + A @ X
                    x = x + B @ y
                    X = X + B @ Y
                xn = np.linalg.norm(x, axis=1)
                zp = np.array([(X[i] - Enew[i] * x[i]) / xn[i] for i in range(2)])  # S126, S128
                dz = np.linalg.norm(zp[0])
                reason = ""
                if dE < o.eps0 and dz < o.r0:                                    # S127
                    conv = True
                    reason = "converged"
                else:
                    reason = restart_reason_after_update(t, dz, o)
                if record:
                    steps.append(PairStep(alpha, seg, t, Enew[0], Enew[1], dE, dz, reason,
                                          B[0, 0], B[1, 1], kn[0], kn[1]))
                E = Enew
                if conv:
                    break
                if reason:
                    # restart: normalised x's (and X's), E_0 = E_{t+1}; back to the
                    # segment start
                    x, X = x / xn[:, None], X / xn[:, None]
                    seg += 1
                    break
                if nstep >= o.max_steps:
                    break
                t += 1
            if nstep >= o.max_steps and not conv:
                all_conv = False
                break
        xn = np.linalg.norm(x, axis=1)
        xc.append(x[0] / xn[0])                   # state alpha accepted
        Xcs.append(X[0] / xn[0])
        Ec.append(float(E[0]))
        # next pair: the converged partner, and the next start vector of Eq. S75
        xa, Xa = x[1] / xn[1], X[1] / xn[1]
        if alpha + 2 < nroots:
            xb, Xb = xs[alpha + 2].copy(), Xs[alpha + 2].copy()
            # Section S2.2: orthogonalise against the converged roots and x_0^alpha
            Xc = np.array(xc)
            proj = Xc @ xb
            xb = xb - Xc.T @ proj
            Xb = Xb - images().T @ proj
            pa = xa @ xb
            xb = xb - pa * xa
            Xb = Xb - pa * Xa
    # the highest state with SBCI1 (Fig. 1B), from the last partner
    Ea = float(xa @ Xa / (xa @ xa))
    prev = (xc, Ec, xa, Xa, Ea, Xcs if o.s78_images else None)
    r1 = S1.sbci1(op, diag, nroots, o, record=False, prev=prev)
    return Result2(r1.energies, r1.vectors, nsig + r1.nsigma, steps, all_conv and r1.converged)
