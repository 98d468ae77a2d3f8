"""SBCI1 and block-Davidson references in FP64 NumPy (oracle; test infrastructure only).

SBCI1 follows Algorithm 1 and Supplementary Sections S1.1-S1.5 step by step,
in the paper's notation:

* start vectors: n lowest diagonal elements -> unit vectors, H in that
  subspace diagonalised (Eqs. S1-S3); or a caller-supplied x0;
* per root alpha: project the start vector off the converged roots and
  normalise (Eqs. S4-S7, the root start of Algorithm 1);
* a segment starts with y = Y = 0, b0 = 1, z'0 = (H - E0) x0;
* each step: z = (1 - sum x_c x_c^T)(D - E^0)^-1 z'   (Eq. S31 / S8),
  Z = H z (Eq. S32, the only sigma per step); t = 0 uses the 2x2 problem
  V_0 (Eqs. S10-S24), t >= 1 the 3x3 problem V_t (Eqs. S33-S55);
  y <- y - c z, Y <- Y - c Z, x <- x + b y, X <- X + b Y (Eqs. S25-S28,
  S56-S59); z' = (X - E x) / |x| (Algorithm 1's residual);
* convergence dE < eps0 and |z'| < r0 (Eqs. S30/S61); otherwise restart on
  Eq. S62a, S62b, S62c or when max_cycle steps were taken (Section S1.5);
* the next root starts from the second Ritz vector of the converging step
  (Section S1.4).

Readings of points the paper leaves open:
  residual scale (the z' of Algorithm 1's residual, positive 1/|x|);
  preconditioner shift E^0 = current energy for the ground state, E_c^0
  for excited roots; |D - E^0| floored at 1e-8; max_cycle per segment;
  a vanishing Gram-Schmidt radicand or Ritz coefficient restarts the
  segment from the Ritz vector; ties in the lowest diagonal elements are
  broken by the lower index.

Davidson: block Davidson-Liu (the paper's baseline), block = nroots,
preconditioner (D - theta_k)^-1 per root with the same floor, two-pass
Gram-Schmidt, max_space = 12 + nroots, collapse to the Ritz vectors.
parity unpinned: Davidson's trajectory; only its converged eigenpairs are
pinned (to eigh/eigsh).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Options:
    eps0: float = 1e-10     # energy threshold (Eq. S30/S61, frozen core = No)
    r0: float = 1e-5        # residual threshold
    b_th: float = 1e-2      # Eq. S62a
    eps1: float = 1e-7      # Eq. S62a
    x_th1: float = 0.1      # Eq. S62b
    x_th2: float = 1.2      # Eq. S62b
    r1: float = 1.0         # Eq. S62c
    max_cycle: int = 20     # Section S1.5
    max_steps: int = 2000   # per root (sigma builds)
    precond_floor: float = 1e-8
    lindep: float = 1e-14   # canonical-orthogonalisation cut-off reused as the rank guard
    max_space_extra: int = 12


@dataclass
class StepRecord:
    root: int
    segment: int
    t: int
    E: float
    dE: float
    dz: float
    b: float
    c: float
    xnorm: float
    reason: str


@dataclass
class Result:
    energies: np.ndarray
    vectors: np.ndarray
    nsigma: int
    steps: list = field(default_factory=list)
    converged: bool = True


def restart_reason(alpha, t, b, dE, xn, dz, o: Options) -> str:
    """Section S1.5: why the segment restarts after step t of root alpha, or "".

    b = b_t, dE = |E_{t+1} - E_t|, xn = |x_{t+1}| (= |k_t|), dz = |z'_{t+1}|.
    Tested in the paper's order: Eq. S62a (excited roots only: a stalled b
    with a settled energy), Eq. S62b (the norm left [x_th1, x_th2]), Eq. S62c
    (a large residual, not on a segment's first step), then max_cycle steps
    in the segment.  Comparisons are strict."""
    if alpha > 0 and abs(b) < o.b_th and dE < o.eps1:
        return "S62a"
    if xn < o.x_th1 or xn > o.x_th2:
        return "S62b"
    if dz > o.r1 and t > 0:
        return "S62c"
    if t + 1 == o.max_cycle:
        return "max_cycle"
    return ""


def start_vectors(op, diag, n):
    """Section S1.1: n lowest diagonal determinants, H diagonalised in their span."""
    ndet = diag.shape[0]
    order = np.lexsort((np.arange(ndet), diag))[:n]
    xs = np.zeros((n, ndet))
    xs[np.arange(n), order] = 1.0       # distinct unit vectors: Gram-Schmidt keeps all
    Xs = np.atleast_2d(op(xs))
    Hs = xs @ Xs.T
    Hs = 0.5 * (Hs + Hs.T)
    E, U = np.linalg.eigh(Hs)
    x0 = U.T @ xs                        # Eq. S2
    X0 = U.T @ Xs                        # Eq. S3
    return x0, X0, E


def ritz_first(Nxx, Nxz, Nzz, Hxx, Hxz, Hzz, lindep):
    """2x2 problem of the first step of a segment (Eqs. S10-S24), |x0| = 1."""
    rad = Nzz - Nxz * Nxz
    if not rad > lindep * max(Nzz, 1e-300):
        return None
    Bz = 1.0 / np.sqrt(rad)                       # S12
    Bx = -Nxz * Bz                                # S13
    V = np.array([[Hxx, Bx * Hxx + Bz * Hxz],     # S15a, S15b
                  [Bx * Hxx + Bz * Hxz, Bx * Bx * Hxx + Bz * Bz * Hzz + 2 * Bx * Bz * Hxz]])
    w, v = np.linalg.eigh(V)
    # coefficients of each Ritz vector on (x, y, z), Eq. S17
    coef = np.array([[v[0, i] + v[1, i] * Bx, 0.0, v[1, i] * Bz] for i in range(2)])
    den = coef[0, 0]
    if abs(den) < lindep:
        return dict(E=w, coef=coef, ok=False)
    k = 1.0 / den                                 # S23
    c = -v[1, 0] * Bz / den                       # S24
    return dict(E=w, coef=coef, ok=True, b=1.0, c=c, k=k)


def ritz_next(N, Hm, lindep):
    """3x3 problem of a later step (Eqs. S33-S55).  N, Hm: dicts of the 6 dots each."""
    Nxx, Nxy, Nxz, Nyy, Nyz, Nzz = (N[k] for k in ("xx", "xy", "xz", "yy", "yz", "zz"))
    Hxx, Hxy, Hxz, Hyy, Hyz, Hzz = (Hm[k] for k in ("xx", "xy", "xz", "yy", "yz", "zz"))
    Ax = 1.0 / np.sqrt(Nxx)                        # S34
    rady = Nyy - Nxy * Nxy / Nxx
    if not rady > lindep * max(Nyy, 1e-300):
        return None
    By = 1.0 / np.sqrt(rady)                       # S36
    Bx = -(Nxy / Nxx) * By                         # S37
    P = Bx * Nxz + By * Nyz                        # S42
    radz = Nzz - Nxz * Nxz / Nxx - P * P
    if not radz > lindep * max(Nzz, 1e-300):
        return None
    Cz = 1.0 / np.sqrt(radz)                       # S39
    Cy = -P * By * Cz                              # S40
    Cx = -(Nxz / Nxx + P * Bx) * Cz                # S41
    vxx = Ax * Ax * Hxx                                                    # S44a
    vxy = Ax * (Bx * Hxx + By * Hxy)                                       # S44b
    vxz = Ax * (Cx * Hxx + Cy * Hxy + Cz * Hxz)                            # S44c
    vyy = Bx * Bx * Hxx + By * By * Hyy + 2 * Bx * By * Hxy                # S44d
    vyz = Bx * (Cx * Hxx + Cy * Hxy + Cz * Hxz) + By * (Cx * Hxy + Cy * Hyy + Cz * Hyz)  # S44e
    vzz = (Cx * Cx * Hxx + Cy * Cy * Hyy + Cz * Cz * Hzz
           + 2 * Cx * Cy * Hxy + 2 * Cx * Cz * Hxz + 2 * Cy * Cz * Hyz)    # S44f
    V = np.array([[vxx, vxy, vxz], [vxy, vyy, vyz], [vxz, vyz, vzz]])
    w, v = np.linalg.eigh(V)
    coef = np.array([[v[0, i] * Ax + v[1, i] * Bx + v[2, i] * Cx,          # S46
                      v[1, i] * By + v[2, i] * Cy,
                      v[2, i] * Cz] for i in range(3)])
    kden = coef[0, 0]
    bden = coef[0, 1]
    if abs(kden) < lindep or abs(bden) < lindep:
        return dict(E=w, coef=coef, ok=False)
    k = 1.0 / kden                                 # S53
    b = bden / kden                                # S54
    c = -v[2, 0] * Cz / bden                       # S55
    return dict(E=w, coef=coef, ok=True, b=b, c=c, k=k)


def sbci1(op, diag, nroots, opts: Options | None = None, x0=None, record=True, prev=None):
    """Lowest nroots eigenpairs of H by SBCI1 (Algorithm 1).  op(v) = H v.

    prev = (x_c list, E_c list, x0, X0, E0[, images]): continue after len(x_c)
    converged roots from the start vector x0 (X0 = H x0), as SBCI2 does for
    its last state (Fig. 1B).  images, if given and not None, are H x_c of
    those roots and replace E_c x_c in Eq. S5 for them."""
    o = opts or Options()
    diag = np.asarray(diag, dtype=np.float64)
    ndet = diag.shape[0]
    nsig = 0
    first = 0
    if prev is not None:
        xc0, Ec0, xa, Xa, Ea = prev[:5]
        first = len(xc0)
        xa, Xa, Ea = np.array(xa, dtype=np.float64), np.array(Xa, dtype=np.float64), float(Ea)
    elif x0 is None:
        xs, Xs, Es = start_vectors(op, diag, nroots)
        nsig += nroots
        xa, Xa, Ea = xs[0].copy(), Xs[0].copy(), float(Es[0])
    else:
        xa = np.asarray(x0, dtype=np.float64).copy()
        xa /= np.linalg.norm(xa)
        Xa = op(xa)
        nsig += 1
        Ea = float(xa @ Xa)
    xc, Ec = ([], []) if prev is None else (list(prev[0]), list(prev[1]))
    Hxc = [] if prev is None or len(prev) < 6 or prev[5] is None else list(prev[5])
    steps = []
    all_conv = True

    for alpha in range(first, nroots):
        # the root start of Algorithm 1 (Eqs. S4-S7)
        if xc:
            Xc = np.array(xc)
            proj = Xc @ xa
            xa = xa - Xc.T @ proj
            # Eq. S5: E_c x_c stands for H x_c, except where H x_c is given
            img = np.array([Hxc[i] if i < len(Hxc) else Ec[i] * xc[i] for i in range(len(xc))])
            Xa = Xa - img.T @ proj
        nrm = np.linalg.norm(xa)
        x, X, E = xa / nrm, Xa / nrm, Ea
        seg = 0
        nstep = 0
        conv = False
        second = None
        while not conv:
            # segment start
            y = np.zeros(ndet)
            Y = np.zeros(ndet)
            zp = X - E * x
            t = 0
            while True:
                E0 = E if alpha == 0 else Ec[0]
                den = diag - E0
                den = np.where(np.abs(den) < o.precond_floor, o.precond_floor, den)
                w = zp / den
                if xc:
                    Xc = np.array(xc)
                    z = w - Xc.T @ (Xc @ w)                   # Eq. S31
                else:
                    z = w
                Z = op(z)                                     # Eq. S32
                nsig += 1
                nstep += 1
                if t == 0:
                    r = ritz_first(x @ x, x @ z, z @ z, x @ X, x @ Z, z @ Z, o.lindep)
                else:
                    N = dict(xx=x @ x, xy=x @ y, xz=x @ z, yy=y @ y, yz=y @ z, zz=z @ z)
                    Hm = dict(xx=x @ X, xy=x @ Y, xz=x @ Z, yy=y @ Y, yz=y @ Z, zz=z @ Z)
                    r = ritz_next(N, Hm, o.lindep)
                if r is None or not r["ok"]:
                    if r is None:
                        # rank-deficient subspace: restart from normalised x
                        if t == 0:
                            raise FloatingPointError("SBCI1: z in span{x} at a segment start")
                        reason = "rank"
                        nx = np.linalg.norm(x)
                        x, X = x / nx, X / nx
                    else:
                        cf = r["coef"][0]
                        v = cf[0] * x + cf[1] * y + cf[2] * z
                        V = cf[0] * X + cf[1] * Y + cf[2] * Z
                        nv = np.linalg.norm(v)
                        x, X, E = v / nv, V / nv, float(r["E"][0])
                        reason = "coef"
                    if record:
                        steps.append(StepRecord(alpha, seg, t, E, np.nan, np.nan, np.nan,
                                                np.nan, 1.0, reason))
                    seg += 1
                    break
                Enew = float(r["E"][0])
                b, c = r["b"], r["c"]
                coef2 = r["coef"][1]
                zt, Zt = z, Z
                y = y - c * z
                Y = Y - c * Z
                x = x + b * y
                X = X + b * Y
                xn = np.linalg.norm(x)
                zp = (X - Enew * x) / xn
                dE = abs(Enew - E)
                dz = np.linalg.norm(zp)
                if dE < o.eps0 and dz < o.r0:
                    xc.append(x / xn)
                    Ec.append(Enew)
                    # Section S1.4: second Ritz vector, written in x_{t+1}, y_{t+1}, z_t
                    ax, ay, az = coef2
                    v = ax * (x - b * y) + ay * (y + c * zt) + az * zt
                    V = ax * (X - b * Y) + ay * (Y + c * Zt) + az * Zt
                    second = (v, V, float(r["E"][1]))
                    conv = True
                    reason = "converged"
                else:
                    reason = restart_reason(alpha, t, b, dE, xn, dz, o)
                if record:
                    steps.append(StepRecord(alpha, seg, t, Enew, dE, dz, b, c, xn, reason))
                E = Enew
                if conv:
                    break
                if reason:
                    x, X = x / xn, X / xn
                    seg += 1
                    break
                if nstep >= o.max_steps:
                    break
                t += 1
            if nstep >= o.max_steps and not conv:
                all_conv = False
                xc.append(x / np.linalg.norm(x))
                Ec.append(E)
                break
        if alpha + 1 < nroots:
            if second is None:
                raise FloatingPointError("SBCI1: no start vector for the next root")
            xa, Xa, Ea = second
    return Result(np.array(Ec), np.array(xc), nsig, steps, all_conv)


def davidson(op, diag, nroots, opts: Options | None = None):
    """Block Davidson-Liu reference (the paper's baseline method)."""
    o = opts or Options()
    diag = np.asarray(diag, dtype=np.float64)
    ndet = diag.shape[0]
    max_space = o.max_space_extra + nroots
    order = np.lexsort((np.arange(ndet), diag))[:nroots]
    V = np.zeros((nroots, ndet))
    V[np.arange(nroots), order] = 1.0
    W = np.atleast_2d(op(V))
    nsig = nroots
    theta_old = np.full(nroots, np.inf)
    for it in range(o.max_steps):
        Hs = V @ W.T
        Hs = 0.5 * (Hs + Hs.T)
        th, U = np.linalg.eigh(Hs)
        th, U = th[:nroots], U[:, :nroots]
        X = U.T @ V
        R = U.T @ W - th[:, None] * X
        rn = np.linalg.norm(R, axis=1)
        dE = np.abs(th - theta_old)
        conv = (dE < o.eps0) & (rn < o.r0)
        theta_old = th
        if conv.all():
            return Result(th, X, nsig, [], True)
        new = []
        for k in np.nonzero(~conv)[0]:
            den = diag - th[k]
            den = np.where(np.abs(den) < o.precond_floor, o.precond_floor, den)
            new.append(R[k] / den)
        if V.shape[0] + len(new) > max_space:
            V, W = X, U.T @ W
        basis = list(V)
        add = []
        for v in new:
            for _ in range(2):
                for b in basis + add:
                    v = v - (b @ v) * b
            nv = np.linalg.norm(v)
            if nv > o.lindep ** 0.5:
                add.append(v / nv)
        if not add:
            return Result(th, X, nsig, [], False)
        A = np.array(add)
        WA = np.atleast_2d(op(A))
        nsig += A.shape[0]
        V = np.vstack([V, A])
        W = np.vstack([W, WA])
    return Result(th, X, nsig, [], False)
