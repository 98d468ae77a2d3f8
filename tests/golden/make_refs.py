"""Write tests/golden/refs.json: reference energies computed by the oracle only.

Run:  python tests/golden/make_refs.py
Contents (all FP64, electronic energies, Eh):
  cas6   seed 0, rank 12: dense Slater-Condon eigh (lowest 6) and the oracle
         SBCI1 energy from the start e_0 + 1e-3 * noise (one root);
  cas10  seeds 0..9, rank 20: Lanczos eigsh on the oracle sigma (lowest 6,
         tol 1e-14), oracle SBCI1 (3 roots, Section S1.1 start) and oracle
         Davidson (3 roots).
  batch512  every 32nd instance of the 512-instance batching workload
         (master seed 2603): oracle SBCI1 with that instance's roots and
         the lowest eigenvalues from Lanczos eigsh on the oracle sigma.

  sbci2  oracle SBCI2 (Algorithm 2) energies: CAS(10,10) seeds 0..2 with 3
         roots, rank 20.
  cas14  CAS(14e,14o), seed 0, rank 28 (11,778,624 determinants): oracle
         SBCI1 with 5 roots (Section S1.1 start, Section S1.4 sequencing;
         eps0 = 1e-10, r0 = 1e-5) and the lowest 6 eigenvalues from Lanczos
         eigsh on the oracle sigma (tol 1e-12).  About 400 oracle sigma calls
         (roughly 2.5 h on 8 cores); the section is written after each part.

"python tests/golden/make_refs.py batch" (or "sbci2", "cas14") recomputes
only that section.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from scipy.sparse.linalg import LinearOperator, eigsh  # noqa: E402

from oracle import hamiltonian as H  # noqa: E402
from oracle import sbci  # noqa: E402
from oracle import sbci2  # noqa: E402
from oracle import sigma as S  # noqa: E402
from workloads import batch_instances, make_integrals, start_noise  # noqa: E402

REFS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "refs.json")
BATCH_SAMPLE = list(range(0, 512, 32))


def batch_section():
    sec = {}
    inst = batch_instances(512, 2603)
    for i in BATCH_SAMPLE:
        t = time.time()
        n, m, nroots, seed = inst[i]
        I = make_integrals(n, 2 * n, seed)
        op = S.Operator(n, m, m, I.h1, I.eri)
        L = LinearOperator((op.ndet, op.ndet), matvec=lambda v: S.sigma(n, m, m, I.h1, I.eri, v),
                           dtype=np.float64)
        ev = np.sort(eigsh(L, k=min(6, op.ndet - 1), which="SA", tol=1e-14)[0])
        rs = sbci.sbci1(op, op.diag(), nroots)
        sec[str(i)] = {"norb": n, "nelec": m, "nroots": nroots, "seed": seed, "rank": 2 * n,
                       "eigsh": ev.tolist(), "sbci1": rs.energies.tolist(), "digest": I.digest()}
        print("batch", i, n, nroots, rs.energies, f"{time.time() - t:.1f}s", flush=True)
    return sec


def sbci2_section():
    sec = {}
    for seed in range(3):
        t = time.time()
        I = make_integrals(10, 20, seed)
        op = S.Operator(10, 5, 5, I.h1, I.eri)
        r = sbci2.sbci2(op, op.diag(), 3)
        sec[str(seed)] = {"sbci2": r.energies.tolist(), "nsigma": r.nsigma, "converged": r.converged,
                          "digest": I.digest()}
        print("sbci2", seed, r.energies, f"{time.time() - t:.1f}s", flush=True)
    return sec


def cas14_section(save):
    """CAS(14,14): oracle SBCI1 (5 roots), then eigsh; save(sec) after each."""
    n, na, nb, K, nroots = 14, 7, 7, 28, 5
    I = make_integrals(n, K, 0)
    op = S.Operator(n, na, nb, I.h1, I.eri)
    sec = {"norb": n, "nalpha": na, "nbeta": nb, "rank": K, "seed": 0, "nroots": nroots,
           "digest": I.digest()}
    t = time.time()
    rs = sbci.sbci1(op, op.diag(), nroots)
    sec.update({"sbci1": rs.energies.tolist(), "sbci1_nsigma": rs.nsigma,
                "sbci1_converged": bool(rs.converged),
                "sbci1_resid": [float(s.dz) for s in rs.steps if s.reason == "converged"],
                "sbci1_seconds": round(time.time() - t, 1)})
    print("cas14 sbci1", rs.energies, rs.nsigma, f"{time.time() - t:.0f}s", flush=True)
    save(sec)
    t = time.time()
    cnt = [0]

    def mv(v):
        cnt[0] += 1
        return S.sigma(n, na, nb, I.h1, I.eri, v)
    L = LinearOperator((op.ndet, op.ndet), matvec=mv, dtype=np.float64)
    ev = np.sort(eigsh(L, k=6, which="SA", tol=1e-12, ncv=24)[0])
    sec.update({"eigsh": ev.tolist(), "eigsh_nsigma": cnt[0],
                "eigsh_seconds": round(time.time() - t, 1)})
    print("cas14 eigsh", ev, cnt[0], f"{time.time() - t:.0f}s", flush=True)
    save(sec)
    return sec


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("batch", "sbci2", "cas14"):
        with open(REFS) as f:
            out = json.load(f)

        def save(sec):
            out[sys.argv[1]] = sec
            with open(REFS, "w") as f:
                json.dump(out, f, indent=1)
        if sys.argv[1] == "batch":
            save(batch_section())
        elif sys.argv[1] == "sbci2":
            save(sbci2_section())
        else:
            cas14_section(save)
        return
    out = {"generator": "tests/golden/make_refs.py", "cas6": {}, "cas10": {}}
    n, na, nb, K = 6, 3, 3, 12
    I = make_integrals(n, K, 0)
    Hs = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    w = np.linalg.eigvalsh(Hs)
    op = S.Operator(n, na, nb, I.h1, I.eri)
    x0 = np.zeros(op.ndet)
    x0[0] = 1.0
    x0 = x0 + 1e-3 * start_noise(n, K, 0, op.ndet)
    r = sbci.sbci1(op, op.diag(), 1, x0=x0)
    out["cas6"] = {"seed": 0, "rank": K, "eigh": w[:6].tolist(), "sbci1": r.energies.tolist(),
                   "sbci1_nsigma": r.nsigma, "digest": I.digest()}
    for seed in range(10):
        t = time.time()
        n, na, nb, K = 10, 5, 5, 20
        I = make_integrals(n, K, seed)
        op = S.Operator(n, na, nb, I.h1, I.eri)
        L = LinearOperator((op.ndet, op.ndet), matvec=lambda v: S.sigma(n, na, nb, I.h1, I.eri, v),
                           dtype=np.float64)
        ev = np.sort(eigsh(L, k=6, which="SA", tol=1e-14)[0])
        d = op.diag()
        rs = sbci.sbci1(op, d, 3)
        rd = sbci.davidson(op, d, 3)
        out["cas10"][str(seed)] = {"rank": K, "eigsh": ev.tolist(), "sbci1": rs.energies.tolist(),
                                   "sbci1_nsigma": rs.nsigma, "davidson": rd.energies.tolist(),
                                   "davidson_nsigma": rd.nsigma, "digest": I.digest()}
        print(seed, ev[:3], rs.energies, rd.energies, f"{time.time() - t:.1f}s", flush=True)
    out["batch512"] = batch_section()
    out["sbci2"] = sbci2_section()
    with open(REFS, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
