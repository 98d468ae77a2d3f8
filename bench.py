#!/usr/bin/env python3
"""Benchmark of the SBCI sigma/solve hot path on one MI355X.

One step = one pass of the whole path on the workload, in the paper's
precision: build the context (strings, excitation tables, same-spin lists,
diagonal) from the integrals already on the host, then solve the lowest
nroots states with FP64 SBCI1 to the paper's thresholds (eps0 = 1e-10,
r0 = 1e-5), so every root is within 1e-8 Eh.  The default workload is
CAS(16e,16o), 165,636,900 determinants, ground state.

Reported (one JSON line):
  value          FP64 sigma determinant-applications per second over the
                 whole timed step (N_det x sigma calls / step time), Gdet/s
                 per root (one vector per sigma call);
  ms_per_step    time of one step: FP64 time to |dE| < 1e-8 Eh;
  time_to_1e8_s  FP64 (median of the timed steps) against the precision
                 forms (BF16 ladder, FP32 ladder; median of 3 each, same step);
  sigma          per-dtype sigma throughput and per-kernel durations, HIP
                 events on the library's stream;
  roofline       the step's dominant kernel against the MI355X peak;
  roofline_same  the same-spin list kernel (ALU and LDS figures);
  cas14          CAS(14e,14o), 5 roots: FP64, both precision forms and SBCI2,
                 each root's energy against the oracle's (tests/golden);
  batch, cas6, cas10, dilute45, symmetry   the other workloads;
  cpu_baseline   the CPU oracle's FP64 string sigma on the host cores, on a
                 bounded sample of determinant rows;
  oracle_checks  from the same oracle rows: the GPU sigma's relative error per
                 dtype, and the GPU ground state's residual on sampled rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks; LDS: 128 B/clk/CU x 256 CUs x 2.4 GHz
    "f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12, "lds": 78.6e12,
}


def note(msg):
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cas16",
                    choices=["cas6", "cas10", "cas14", "cas16", "dilute45", "cas14_sym", "cas16_sym"])
    ap.add_argument("--precision", default="bf16", choices=["f64", "f32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sigma-reps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true", help="skip the batching-form section")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the cas6 / cas10 / cas16 sections")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="run only the solver comparison on dilute45 with 6 roots (the shape of "
                         "the paper's CAS(6e,45o) excited-state instance; several minutes) and "
                         "print it")
    ap.add_argument("--solve-driver", choices=["sbci1", "sbci2", "davidson"], default=None,
                    help="profiling driver: one FP64 solve of the workload with this solver; print "
                         "its report and exit")
    ap.add_argument("--only-sym", action="store_true",
                    help="print only the point-group blocked section")
    ap.add_argument("--only-batch", action="store_true",
                    help="profiling driver: run only the batching-form section and print it")
    ap.add_argument("--kernel-driver", choices=["f64", "f32", "bf16"], default=None,
                    help="profiling driver: run --sigma-reps sigma calls of this dtype on the "
                         "workload and one 1 GiB device copy (the counter scale reference), "
                         "print their sizes and exit")
    return ap.parse_args()


def roofline(cfg, ndet, kname, kdt, k_ms):
    """Roofline of one sigma part for one launch (one vector) of the workload.

    opp_mfma: MFMA-bound; algorithmic flops = 2 s^2 per determinant (the
      minimum count of the D * (pq|rs) * E contraction); the row-stationary
      MFMA form issues 2 npair s (reported as issue_frac).
    same_*:   bound by arithmetic on gathered operands ("alu"); algorithmic
      flops = 2 F per determinant (F same-spin list entries per string).
    transpose / add_t: HBM-bound; 2 (or 3) vector passes.
    """
    n, m = cfg["norb"], cfg["na"]
    s = m * (n - m + 1)
    npair = n * (n + 1) // 2
    nf = 1 + m * (n - m) + comb(m, 2) * comb(n - m, 2)
    esz = 8 if kdt == "f64" else 4
    t = k_ms / 1e3
    if kname == "opp_mfma":
        r = {"bound": "mfma", "achieved": 2.0 * s * s * ndet / t / 1e12, "peak": PEAK[kdt] / 1e12,
             "unit": "TFLOP/s"}
        r["issue_frac"] = 2.0 * npair * s * ndet / t / PEAK[kdt]
    elif kname.startswith("same"):
        vpk = PEAK["f64"] if kdt == "f64" else PEAK["f32"]
        r = {"bound": "alu", "achieved": 2.0 * nf * ndet / t / 1e12, "peak": vpk / 1e12,
             "unit": "TFLOP/s"}
        # the list kernels read one source element from LDS per list entry
        # and column: nf * element bytes per determinant
        r["lds_achieved_TBps"] = nf * esz * ndet / t / 1e12
        r["lds_peak_TBps"] = PEAK["lds"] / 1e12
        r["lds_frac"] = r["lds_achieved_TBps"] / r["lds_peak_TBps"]
    else:
        passes = 3.0 if kname == "add_t" else 2.0
        r = {"bound": "hbm", "achieved": passes * esz * ndet / t / 1e9, "peak": PEAK["hbm"] / 1e9,
             "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    meas = measured(kname, kdt, cfg)
    r["traffic"] = meas.get("traffic_bytes_per_launch")
    if kname == "opp_mfma":
        r["mfma_busy"] = meas.get("mfma_busy")
    r["kernel"] = f"{kname} ({kdt})"
    r["ms_per_launch"] = k_ms
    return r


KERNEL_SOURCE = {"opp_mfma": "sigma.hip", "same_alpha": "sigma.hip", "same_beta": "sigma.hip",
                 "transpose": "sigma.hip", "add_t": "sigma.hip", "opp_orbital": "sigma.hip",
                 "same_dense": "sigma.hip"}


def kernel_text_sha(path, func):
    """SHA-256 of one kernel's definition in a source file: from its
    template line to the closing brace at column 0 (comments above it are
    not part of it).  Counter figures stay valid while this text is
    unchanged, whatever else the file gains."""
    import hashlib
    import re
    lines = open(path).read().split("\n")
    i = next((k for k, ln in enumerate(lines) if re.search(r"\bvoid " + func + r"\(", ln)), None)
    if i is None:
        return ""
    j = i
    while j > 0 and not lines[j].startswith("template"):
        if lines[j - 1].strip() == "" or lines[j - 1].startswith("//"):
            break
        j -= 1
    k = i
    while k < len(lines) and lines[k] != "}":
        k += 1
    return hashlib.sha256("\n".join(lines[j:k + 1]).encode()).hexdigest()


def measured(kname, kdt, cfg):
    """Counter figures from the committed rocprofv3 --pmc summary of this
    kernel and workload: HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled
    by a plain copy of known size) and, for the contraction, the MFMA busy
    fraction.  Empty if there is no summary or the kernel source has changed
    since the counters were taken."""
    import hashlib
    name = f"pmc_{kname}_{kdt}_{cfg['name']}.md"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.split()[0].strip("`") if v.split() else ""
    src = os.path.join(ROOT, "paper_2603_06101_amd", "csrc", KERNEL_SOURCE[kname])
    if "kernel_sha256" in fields and "kernel" in fields:
        if fields["kernel_sha256"] != kernel_text_sha(src, fields["kernel"]):
            return {}
    elif fields.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "mfma_busy"):
        try:
            out[key] = float(fields[key])
        except (KeyError, ValueError):
            pass
    return out


def small_sections(sb, stream):
    """cas6: launch-latency regime (us per sigma and per step, noise start);
    cas10 seeds 0..9: FP64 SBCI1 vs Davidson on the same sigma (time, sigma
    calls, peak vector bytes)."""
    import numpy as np
    import torch

    from workloads import CONFIGS, make_integrals, start_noise
    out = {}
    c6 = CONFIGS["cas6"]
    I = make_integrals(c6["norb"], c6["rank"], c6["seed"])
    ctx = sb.Context(6, 3, 3, I.h1, I.eri, stream=stream)
    x0 = np.zeros(ctx.ndet)
    x0[0] = 1.0
    x0 = x0 + 1e-3 * start_noise(6, c6["rank"], c6["seed"], ctx.ndet)
    c = torch.from_numpy(x0).cuda()
    o = ctx.sigma(c)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(200):
        ctx.sigma(c, out=o)
    torch.cuda.synchronize()
    us_sigma = (time.perf_counter() - t) / 200 * 1e6
    ctx.solve(1, tol=1e-10, x0=x0, want_vectors=False)
    r = ctx.solve(1, tol=1e-10, x0=x0, want_vectors=False)
    ref = refs_section("cas6", I.digest())
    out["cas6"] = {"ndet": ctx.ndet, "us_per_sigma": round(us_sigma, 1),
                   "solve_ms": round(r.report["seconds"] * 1e3, 2), "steps": r.report["nsteps"],
                   "us_per_step": round(r.report["seconds"] / max(1, r.report["nsteps"]) * 1e6, 1),
                   "energy": float(r.energies[0]),
                   # the start e_0 + noise is spin-flip symmetric: SBCI1 reaches
                   # the lowest singlet, which lies above a triplet here
                   "oracle_sbci1_energy": (ref.get("sbci1") or [None])[0],
                   "oracle_eigh_lowest": (ref.get("eigh") or [None])[0]}
    ctx.close()
    rows = []
    for seed in range(10):
        I = make_integrals(10, 20, seed)
        ctx = sb.Context(10, 5, 5, I.h1, I.eri, stream=stream)
        if seed == 0:
            ctx.solve(3, tol=1e-10, want_vectors=False)
        s1 = ctx.solve(3, tol=1e-10, want_vectors=False)
        dv = ctx.davidson(3, tol=1e-10, want_vectors=False)
        s2 = ctx.solve2(3, tol=1e-10, want_vectors=False)
        rows.append((s1.report["seconds"], dv.report["seconds"], s1.report["nsigma_f64"],
                     dv.report["nsigma_f64"], s1.report["peak_vector_bytes"],
                     dv.report["peak_vector_bytes"],
                     float(abs(s1.energies[0] - dv.energies[0]) < 1e-8),
                     s2.report["seconds"], s2.report["nsigma_f64"], s2.report["peak_vector_bytes"],
                     float(np.abs(np.sort(s2.energies) - np.sort(dv.energies)).max() < 1e-7)))
        ctx.close()
    a = np.array(rows)
    out["cas10"] = {
        "ndet": 63504, "roots": 3, "seeds": 10,
        "sbci1_ms_median": round(float(np.median(a[:, 0])) * 1e3, 2),
        "davidson_ms_median": round(float(np.median(a[:, 1])) * 1e3, 2),
        "sbci1_sigma_median": float(np.median(a[:, 2])), "davidson_sigma_median": float(np.median(a[:, 3])),
        "sbci1_peak_vector_MB": round(float(np.median(a[:, 4])) / 1e6, 2),
        "davidson_peak_vector_MB": round(float(np.median(a[:, 5])) / 1e6, 2),
        # SBCI1 from the spin-flip-symmetric start can converge to a singlet
        # above a lower odd-S state; Davidson (block start) finds the lowest
        "seeds_sbci1_root0_is_lowest": int(np.sum(a[:, 6])),
        "sbci2_ms_median": round(float(np.median(a[:, 7])) * 1e3, 2),
        "sbci2_sigma_median": float(np.median(a[:, 8])),
        "sbci2_peak_vector_MB": round(float(np.median(a[:, 9])) / 1e6, 2),
        "seeds_sbci2_equals_davidson_roots": int(np.sum(a[:, 10])),
    }
    return out


def cas16_section(sb, stream, precision):
    """cas16 (165,636,900 determinants, ground state): sigma per dtype and the
    time to 1e-8 Eh, mixed vs FP64."""
    import torch

    from workloads import CONFIGS, make_integrals
    cf = CONFIGS["cas16"]
    I = make_integrals(cf["norb"], cf["rank"], cf["seed"])
    t = time.perf_counter()
    ctx = sb.Context(16, 8, 8, I.h1, I.eri, stream=stream)
    torch.cuda.synchronize()
    out = {"ndet": ctx.ndet, "create_s": round(time.perf_counter() - t, 3), "sigma": {}}
    parts = ["same_alpha", "opp_mfma", "transpose", "same_beta", "add_t"]
    c = torch.randn(ctx.ndet, dtype=torch.float32, device="cuda")
    for dt in ("bf16", "f32", "f64"):
        x = c.double() if dt == "f64" else c
        o, _ = ctx.sigma_timed(x, dt)
        o, ms = ctx.sigma_timed(x, dt, out=o)
        out["sigma"][dt] = {"gdet_per_s": round(ctx.ndet / (sum(ms) / 1e3) / 1e9, 3),
                            "kernels_ms": dict(zip(parts, [round(v, 3) for v in ms]))}
        del o, x
    del c
    res = {}
    for prec in (precision, "f64"):
        t = time.perf_counter()
        r = ctx.solve(1, tol=1e-10, opts=dict(precision=prec), want_vectors=False)
        torch.cuda.synchronize()
        res[prec] = (time.perf_counter() - t, r)
    ctx.close()
    tm, rm = res[precision]
    t64, r64 = res["f64"]
    out["time_to_1e8_s"] = {"mixed": round(tm, 3), "fp64": round(t64, 3), "speedup": round(t64 / tm, 3)}
    out["nsigma"] = {"f64": rm.report["nsigma_f64"], "low": rm.report["nsigma_low"],
                     "bf16": rm.report["nsigma_bf16"]}
    out["abs_dE_vs_fp64"] = float(abs(rm.energies[0] - r64.energies[0]))
    out["peak_vector_GB"] = round(rm.report["peak_vector_bytes"] / 1e9, 2)
    return out


def sym_pair_count(norb, na, nb, orbsym, irrep):
    """Multiply-adds of the blocked opposite-spin part: for each determinant of
    the irrep, the pairs (alpha excitation e, beta excitation f) of equal
    class orbsym[p] ^ orbsym[q], summed block by block."""
    from itertools import combinations

    import numpy as np

    def per_irrep(m):
        tot = np.zeros((8, 8))        # [string irrep][class] -> excitations summed over strings
        cnt = np.zeros(8)
        for occ in combinations(range(norb), m):
            g = 0
            for p in occ:
                g ^= int(orbsym[p])
            cnt[g] += 1
            occs = set(occ)
            for q in occ:
                for p in range(norb):
                    if p == q or p not in occs:
                        tot[g][int(orbsym[p]) ^ int(orbsym[q])] += 1
        return tot, cnt

    ta, ca = per_irrep(na)
    tb, cb = per_irrep(nb) if nb != na else (ta, ca)
    pairs = 0.0
    for a in range(8):
        b = a ^ irrep
        for x in range(8):
            pairs += ta[a][x] * tb[b][x]
    return pairs


def sym_section(sb, stream):
    """Point-group blocked workloads (irrep 0 of orbital labels p mod 8, totally
    symmetric integrals): CAS(14e,14o) with 5 roots and CAS(16e,16o) with the
    ground state.  Blocked sigma per dtype (the opposite-spin part in the
    vector pair form, BF16 on MFMA; "f64_class_mfma": the MFMA form in FP64)
    and the time to 1e-8 Eh in FP64 and in the FP32 and BF16 precision
    forms."""
    import statistics

    import numpy as np
    import torch

    from workloads import CONFIGS, make_sym_integrals, orbital_irreps, sigma_inputs
    out = {}
    for name in ("cas14_sym", "cas16_sym"):
        cf = CONFIGS[name]
        o = orbital_irreps(cf["norb"])
        I = make_sym_integrals(cf["norb"], cf["rank"], cf["seed"], o)
        t = time.perf_counter()
        ctx = sb.Context(cf["norb"], cf["na"], cf["nb"], I.h1, I.eri, stream=stream, orbsym=o,
                         irrep=cf["irrep"])
        torch.cuda.synchronize()
        sec = {"ndet": ctx.ndet, "irrep": cf["irrep"], "create_s": round(time.perf_counter() - t, 3),
               "sigma": {}}
        pairs = sym_pair_count(cf["norb"], cf["na"], cf["nb"], o, cf["irrep"])
        c = torch.from_numpy(sigma_inputs(0, 1, ctx.ndet)[0]).cuda()
        for dt in ("bf16", "f32", "f64", "f64_class_mfma"):
            ctx.set_opp_form("class_mfma" if dt == "f64_class_mfma" else "auto")
            x = c if dt.startswith("f64") else c.float()
            y, _ = ctx.sigma_timed(x, dt[:3] if dt != "bf16" else dt)
            runs = []
            for _ in range(5):
                y, ms = ctx.sigma_timed(x, dt[:3] if dt != "bf16" else dt, out=y)
                runs.append(ms)
            same = statistics.median(r[0] for r in runs)
            opp = statistics.median(r[1] for r in runs)
            sec["sigma"][dt] = {"gdet_per_s": round(ctx.ndet / ((same + opp) / 1e3) / 1e9, 3),
                                "kernels_ms": {"same": round(same, 4), "opp": round(opp, 4)},
                                "opp_gflops": round(2 * pairs / (opp / 1e3) / 1e9, 1)}
            del y, x
        ctx.set_opp_form("auto")
        sec["opp_pairs_per_det"] = round(pairs / ctx.ndet, 1)
        del c
        res = {}
        for prec in ("bf16", "f32", "f64"):
            t = time.perf_counter()
            r = ctx.solve(cf["nroots"], tol=1e-10, opts=dict(precision=prec), want_vectors=False)
            torch.cuda.synchronize()
            res[prec] = (time.perf_counter() - t, r)
        ctx.close()
        tm, rm = res["f32"]
        tb, rb = res["bf16"]
        t64, r64 = res["f64"]
        sec["time_to_1e8_s"] = {"mixed_bf16": round(tb, 3), "mixed_f32": round(tm, 3), "fp64": round(t64, 3),
                                "speedup_bf16": round(t64 / tb, 3), "speedup_f32": round(t64 / tm, 3)}
        sec["energies"] = [float(e) for e in r64.energies]
        sec["max_abs_dE_mixed_vs_fp64"] = {
            p: float(np.abs(np.sort(res[p][1].energies) - np.sort(r64.energies)).max()) for p in ("bf16", "f32")}
        sec["nsigma"] = {"fp64_form": r64.report["nsigma_f64"], "f32_form": [rm.report["nsigma_f64"], rm.report["nsigma_low"]],
                         "bf16_form": [rb.report["nsigma_f64"], rb.report["nsigma_low"]]}
        out[name] = sec
    return out


def dilute45_section(sb, stream, precision):
    """dilute45, CAS(6e,45o) (201,356,100 determinants; the shape of the
    paper's few-electrons-in-many-orbitals instances): the sigma forms chosen,
    sigma per dtype with the MFMA rate of its two dominant parts, and the
    ground state to 1e-8 Eh, mixed vs FP64."""
    import torch

    from workloads import CONFIGS, make_integrals
    cf = CONFIGS["dilute45"]
    n, m = cf["norb"], cf["na"]
    I = make_integrals(n, cf["rank"], cf["seed"])
    t = time.perf_counter()
    ctx = sb.Context(n, m, cf["nb"], I.h1, I.eri, stream=stream)
    torch.cuda.synchronize()
    ns, s = comb(n, m), m * (n - m + 1)
    nf = 1 + m * (n - m) + comb(m, 2) * comb(n - m, 2)
    out = {"ndet": ctx.ndet, "create_s": round(time.perf_counter() - t, 3),
           "forms": {"same_spin": ctx.same_form(0), "opposite_spin": ctx.opp_form("f64")},
           "sigma": {}}
    parts = ["same_alpha", "opp_mfma", "transpose", "same_beta", "add_t"]
    c = torch.randn(ctx.ndet, dtype=torch.float32, device="cuda")
    for dt in ("bf16", "f32", "f64"):
        x = c.double() if dt == "f64" else c
        o, _ = ctx.sigma_timed(x, dt)
        o, ms = ctx.sigma_timed(x, dt, out=o)
        out["sigma"][dt] = {
            "gdet_per_s": round(ctx.ndet / (sum(ms) / 1e3) / 1e9, 3),
            "kernels_ms": dict(zip(parts, [round(v, 3) for v in ms])),
            # algorithmic rates: 2 s^2 flops per determinant for the opposite-
            # spin contraction, 2 F (list entries of a string) per determinant
            # and spin for the same-spin part; the dense product issues 2 N_s
            "opp_tflops": round(2 * s * s * ctx.ndet / (ms[1] / 1e3) / 1e12, 1),
            "same_tflops": round(2 * nf * ctx.ndet / (ms[0] / 1e3) / 1e12, 1),
            "same_dense_issue_tflops": round(2 * ns * ctx.ndet / (ms[0] / 1e3) / 1e12, 1),
        }
        del o, x
    del c
    # rooflines of the two MFMA kernels in FP64 (counter figures from the
    # committed summaries while the kernels' text is unchanged)
    cfgd = dict(cf, name="dilute45")
    ms64 = out["sigma"]["f64"]["kernels_ms"]
    # achieved = the method's flops (2 s^2; 2 F for the same-spin part);
    # issue_frac = what the kernel issues (2 N m s; the dense product's 2 N_s)
    for key, kname, flops, issued, t_ms in (
            ("roofline_opp_orbital", "opp_orbital", 2 * s * s * ctx.ndet, 2 * n * cf["nb"] * s * ctx.ndet,
             ms64["opp_mfma"]),
            ("roofline_same_dense", "same_dense", 2 * nf * ctx.ndet, 2 * ns * ctx.ndet, ms64["same_alpha"])):
        ach = flops / (t_ms / 1e3) / 1e12
        meas = measured(kname, "f64", cfgd)
        out[key] = {"bound": "mfma", "achieved": round(ach, 2), "peak": PEAK["f64"] / 1e12,
                    "unit": "TFLOP/s", "frac": round(ach / (PEAK["f64"] / 1e12), 4),
                    "issue_frac": round(issued / (t_ms / 1e3) / PEAK["f64"], 4),
                    "traffic": meas.get("traffic_bytes_per_launch"),
                    "mfma_busy": meas.get("mfma_busy"), "ms_per_launch": t_ms}
    res = {}
    for prec in (precision, "f64"):
        t = time.perf_counter()
        r = ctx.solve(1, tol=1e-10, opts=dict(precision=prec), want_vectors=False)
        torch.cuda.synchronize()
        res[prec] = (time.perf_counter() - t, r)
    ctx.close()
    tm, rm = res[precision]
    t64, r64 = res["f64"]
    out["time_to_1e8_s"] = {"mixed": round(tm, 3), "fp64": round(t64, 3), "speedup": round(t64 / tm, 3)}
    out["nsigma"] = {"f64": rm.report["nsigma_f64"], "low": rm.report["nsigma_low"],
                     "bf16": rm.report["nsigma_bf16"], "fp64_form": r64.report["nsigma_f64"]}
    out["energy"] = float(r64.energies[0])
    out["abs_dE_vs_fp64"] = float(abs(rm.energies[0] - r64.energies[0]))
    out["peak_vector_GB"] = round(rm.report["peak_vector_bytes"] / 1e9, 2)
    torch.cuda.empty_cache()
    return out


def paper_shapes_section(sb, stream, precision):
    """dilute45 with 6 roots, the shape of the paper's CAS(6e,45o) excited-
    state instance: SBCI1 (mixed and FP64), SBCI2 and Davidson on the same
    sigma; time to 1e-8 Eh, sigma applications, peak vector memory and the
    agreement of the roots.  A progress line goes to stderr after each solve."""
    import numpy as np
    import torch

    from workloads import CONFIGS, make_integrals
    cf = CONFIGS["dilute45"]
    nroots = 6
    I = make_integrals(cf["norb"], cf["rank"], cf["seed"])
    ctx = sb.Context(cf["norb"], cf["na"], cf["nb"], I.h1, I.eri, stream=stream)
    out = {"workload": "dilute45", "ndet": ctx.ndet, "nroots": nroots, "solvers": {}}
    runs = (("sbci1_" + precision, lambda: ctx.solve(nroots, tol=1e-10, opts=dict(precision=precision),
                                                     want_vectors=False)),
            ("sbci1_f64", lambda: ctx.solve(nroots, tol=1e-10, opts=dict(precision="f64"),
                                            want_vectors=False)),
            ("sbci2_f64", lambda: ctx.solve2(nroots, tol=1e-10, want_vectors=False)),
            ("davidson_f64", lambda: ctx.davidson(nroots, tol=1e-10, want_vectors=False)))
    energies = {}
    last = [time.perf_counter()]

    def progress(step):
        # a line from the solve's own step records, at most every 20 s
        now = time.perf_counter()
        if now - last[0] >= 20.0:
            last[0] = now
            print(f"paper-shapes:   root {step['root']} step {step['t']} E {step['E']:.10f} "
                  f"|z'| {step['dz']:.2e} at {step['seconds']:.0f} s", file=sys.stderr, flush=True)

    ctx.set_progress(progress)
    for name, fn in runs:
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        energies[name] = np.sort(np.asarray(r.energies))
        out["solvers"][name] = {"seconds": round(dt, 2), "nsigma_f64": r.report["nsigma_f64"],
                                "nsigma_low": r.report.get("nsigma_low", 0),
                                "peak_vector_GB": round(r.report["peak_vector_bytes"] / 1e9, 2),
                                "status": r.status}
        print(f"paper-shapes: {name} {dt:.1f} s", file=sys.stderr, flush=True)
    ctx.close()
    ref = energies["davidson_f64"]
    out["energies_davidson"] = [float(e) for e in ref]
    out["max_abs_dE_vs_davidson"] = {k: float(np.abs(v - ref).max()) for k, v in energies.items()}
    return out


def batch_section(sb, precision):
    """Batching form: 512 uneven instances, one persistent-kernel graph launch per solve,
    in the FP64 form and both mixed forms (each autotuned)."""
    import numpy as np

    from workloads import batch_instances, make_integrals
    inst = batch_instances(512, 2603)
    ints = []
    for n, m, _, seed in inst:
        I = make_integrals(n, 2 * n, seed)
        ints.append((n, m, m, I.h1, I.eri))
    t = time.perf_counter()
    b = sb.Batch(ints)
    t_create = time.perf_counter() - t
    nroots = [x[2] for x in inst]
    out = {"instances": len(inst), "ndet_total": int(sum(b.ndet)),
           "roots_total": int(sum(nroots)), "create_s": round(t_create, 3)}
    res = {}
    for prec in ("f64", "f32", "bf16"):
        best, cands = b.tune(nroots, tol=1e-10, opts=dict(precision=prec))
        r = b.solve(nroots, tol=1e-10, opts=dict(precision=prec))
        rd = b.solve(nroots, tol=1e-10, opts=dict(precision=prec),
                     config=dict(threads=256, wg_per_cu=2, order=0, k_panel=16))
        spans = np.array([d["t_end"] - d["t_start"] for d in r.instances])
        crit = int(np.argmax(spans))
        res[prec] = r
        out[prec] = {
            "makespan_s": round(r.report["seconds"], 4),
            "gdet_per_s": round(r.report["det_sigma"] / r.report["seconds"] / 1e9, 4),
            "converged": int(r.report["ninst_converged"]),
            "nsigma": {"f64": r.report["nsigma_f64"], "low": r.report["nsigma_low"]},
            "steps": r.report["nsteps"],
            "tuned": best,
            "tuned_vs_default": round(rd.report["seconds"] / r.report["seconds"], 3),
            "candidates_ms": [[c["threads"], c["wg_per_cu"], c["order"], c["k_panel"], c["queue_reserve"],
                               round(ms, 1)] for c, ms in cands],
            "critical_instance": {"id": crit, "norb": inst[crit][0], "nroots": inst[crit][2],
                                  "span_s": round(float(spans[crit]), 4),
                                  "steps": r.instances[crit]["nsteps"]},
            "median_instance_span_s": round(float(np.median(spans)), 5),
            "teams": {"instances": r.report["nteams"], "workgroups": r.report["team_workgroups"]},
        }
    # the faster mixed form against FP64
    best = min(("f32", "bf16"), key=lambda p: res[p].report["seconds"])
    e64 = np.array([e[0] for e in res["f64"].energies])
    emx = np.array([e[0] for e in res[best].energies])
    d = emx - e64
    out["mixed_form"] = best
    out["root0_mixed_minus_fp64"] = {"max_abs_same_state": float(np.max(np.abs(d[np.abs(d) < 1e-6]))),
                                     "lower_state_count": int(np.sum(d < -1e-6))}
    out["speedup_mixed_vs_fp64"] = round(res["f64"].report["seconds"] / res[best].report["seconds"], 3)
    b.close()
    return out


def refs_section(name, digest):
    """Stored oracle values for a workload (tests/golden/refs.json, written by
    tests/golden/make_refs.py from the oracle only), if their integral digest
    matches; {} otherwise."""
    path = os.path.join(ROOT, "tests", "golden", "refs.json")
    try:
        sec = json.load(open(path)).get(name, {})
    except (OSError, ValueError):
        return {}
    return sec if sec.get("digest") == digest else {}


def vs_oracle(energies, ref):
    """|E - E_oracle| per root (both sorted ascending)."""
    import numpy as np
    e, r = np.sort(np.asarray(energies)), np.sort(np.asarray(ref))
    k = min(len(e), len(r))
    return [float(v) for v in np.abs(e[:k] - r[:k])]


def cas14_section(sb, stream, reps):
    """cas14 (11,778,624 determinants), 5 roots: FP64 SBCI1 and both precision
    forms (time to 1e-8 Eh, median of reps runs), SBCI2, and each root's
    energy against the oracle's SBCI1 and eigsh values (tests/golden/refs.json)."""
    import statistics

    import numpy as np
    import torch

    from workloads import CONFIGS, make_integrals
    cf = CONFIGS["cas14"]
    I = make_integrals(cf["norb"], cf["rank"], cf["seed"])
    ref = refs_section("cas14", I.digest())
    ctx = sb.Context(cf["norb"], cf["na"], cf["nb"], I.h1, I.eri, stream=stream)
    out = {"ndet": ctx.ndet, "nroots": cf["nroots"], "forms": {}}
    for name, fn in (
            ("sbci1_f64", lambda: ctx.solve(cf["nroots"], tol=1e-10, opts=dict(precision="f64"),
                                            want_vectors=False)),
            ("sbci1_bf16_ladder", lambda: ctx.solve(cf["nroots"], tol=1e-10,
                                                    opts=dict(precision="bf16"), want_vectors=False)),
            ("sbci1_f32_ladder", lambda: ctx.solve(cf["nroots"], tol=1e-10,
                                                   opts=dict(precision="f32"), want_vectors=False)),
            ("sbci2_f64", lambda: ctx.solve2(cf["nroots"], tol=1e-10, want_vectors=False)),
            ("sbci2_f32_ladder", lambda: ctx.solve2(cf["nroots"], tol=1e-10,
                                                    opts=dict(precision="f32"), want_vectors=False))):
        times, r = [], None
        for _ in range(reps if name.startswith("sbci1") else 1):
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        sec = {"time_to_1e8_s": round(statistics.median(times), 4), "runs": len(times),
               "nsigma": {"f64": r.report["nsigma_f64"], "low": r.report.get("nsigma_low", 0),
                          "bf16": r.report.get("nsigma_bf16", 0)},
               "energies": [float(e) for e in r.energies],
               "residuals": [float(v) for v in r.report.get("resid", [])[:cf["nroots"]]]}
        if ref.get("sbci1"):
            sec["abs_dE_vs_oracle_sbci1"] = vs_oracle(r.energies, ref["sbci1"])
        out["forms"][name] = sec
    ctx.close()
    if ref.get("eigsh"):
        out["oracle_eigsh_lowest"] = ref["eigsh"][:cf["nroots"] + 1]
    if ref.get("sbci1"):
        out["oracle_sbci1"] = ref["sbci1"]
    f = out["forms"]
    out["speedup_vs_fp64"] = {k: round(f["sbci1_f64"]["time_to_1e8_s"] / f[k]["time_to_1e8_s"], 3)
                              for k in ("sbci1_bf16_ladder", "sbci1_f32_ladder")}
    return out


def cpu_legs():
    """The other CPU-baseline legs, the oracle as it stands on the host cores:
    SBCI1 and LAPACK eigh at CAS(6,6) (1 root), SBCI1 and Davidson at
    CAS(10,10) seed 0 (3 roots), each timed once (median of 3 for the
    sub-second ones); and the stored CAS(14,14) 5-root oracle SBCI1 run
    (tests/golden/refs.json, timed when the reference was written, on the
    host that wrote it)."""
    import statistics

    import numpy as np

    from oracle import hamiltonian as H
    from oracle import sbci as OSB
    from oracle import sigma as OS
    from workloads import make_integrals, start_noise
    out = {}
    I = make_integrals(6, 12, 0)
    op = OS.Operator(6, 3, 3, I.h1, I.eri)
    x0 = np.zeros(op.ndet)
    x0[0] = 1.0
    x0 = x0 + 1e-3 * start_noise(6, 12, 0, op.ndet)
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        r = OSB.sbci1(op, op.diag(), 1, x0=x0, record=False)
        ts.append(time.perf_counter() - t)
    out["cas6_sbci1_s"] = round(statistics.median(ts), 4)
    Hd = H.dense_h_slater_condon(6, 3, 3, I.h1, I.eri)
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        np.linalg.eigvalsh(Hd)
        ts.append(time.perf_counter() - t)
    out["cas6_eigh_s"] = round(statistics.median(ts), 5)
    I = make_integrals(10, 20, 0)
    op = OS.Operator(10, 5, 5, I.h1, I.eri)
    d = op.diag()
    t = time.perf_counter()
    r = OSB.sbci1(op, d, 3, record=False)
    out["cas10_sbci1_s"] = round(time.perf_counter() - t, 3)
    out["cas10_sbci1_nsigma"] = r.nsigma
    t = time.perf_counter()
    r = OSB.davidson(op, d, 3)
    out["cas10_davidson_s"] = round(time.perf_counter() - t, 3)
    out["cas10_davidson_nsigma"] = r.nsigma
    ref = refs_section("cas14", make_integrals(14, 28, 0).digest())
    if ref.get("sbci1_seconds"):
        out["cas14_sbci1_s_stored"] = ref["sbci1_seconds"]
        out["cas14_sbci1_nsigma_stored"] = ref.get("sbci1_nsigma")
    return out


def oracle_checks(cfg, I, ndet, sb, stream, seconds, xE=None):
    """The CPU-baseline leg: the oracle's FP64 string sigma on a bounded sample
    of determinant rows, timed on the host cores; the same oracle rows then
    check the GPU sigma of that vector in each dtype (relative error on the
    sample) and, if given, the GPU ground state (x, E): max |(H x)[J] - E x[J]|
    over sampled rows J, against max |E x[J]|."""
    import numpy as np
    import torch

    from oracle import sigma as OS
    from workloads import sigma_inputs
    c = sigma_inputs(0, 1, ndet)[0]
    rng = np.random.default_rng(11)
    # calibration: the rate of a 2000-row and a 50000-row call (the oracle
    # lists every string's excitations once per call, a fixed cost)
    ts = []
    for n in (2000, 50000):
        rows = rng.integers(0, ndet, n)
        t = time.perf_counter()
        OS.sigma_rows(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, c, rows)
        ts.append(time.perf_counter() - t)
    per_row = max((ts[1] - ts[0]) / 48000, 1e-9)
    n2 = int(max(2000, min(2e7, seconds / per_row)))
    rows = np.sort(rng.integers(0, ndet, n2))
    t = time.perf_counter()
    want = OS.sigma_rows(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, c, rows)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    base = {"value": n2 / dt / 1e9, "unit": "Gdet/s", "cores": cores, "kind": "oracle",
            "sample": f"{n2} random determinant rows of the FP64 string sigma "
                      f"({cfg['norb']} orbitals, {ndet} determinants), {dt:.1f} s"}
    checks = {"rows": n2, "sigma_rel_err": {}}
    base["legs"] = cpu_legs()
    ctx = sb.Context(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, stream=stream)
    cg = torch.from_numpy(c).cuda()
    idx = torch.from_numpy(rows).cuda()
    for dt_ in ("f64", "f32", "bf16"):
        x = cg if dt_ == "f64" else cg.float()
        got = ctx.sigma(x, dt_)[idx].double().cpu().numpy()
        checks["sigma_rel_err"][dt_] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        del got, x
    ctx.close()
    del cg
    if xE is not None:
        x, E = xE
        xr = x[idx].cpu().numpy()
        hx = OS.sigma_rows(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, x.cpu().numpy(), rows)
        checks["ground_state_residual"] = {"max_abs": float(np.abs(hx - E * xr).max()),
                                           "scale_max_abs_Ex": float(np.abs(E * xr).max()),
                                           "rows": n2}
    torch.cuda.empty_cache()
    return base, checks


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the path runs on one GPU; --gpus must be 1 "
              "(sharding over several GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    import statistics

    import numpy as np
    import torch

    import paper_2603_06101_amd as sb
    from workloads import CONFIGS, make_integrals, sigma_inputs

    cfg = dict(CONFIGS[a.workload], name=a.workload)
    nroots = cfg["nroots"]
    sym = "irrep" in cfg
    if sym:
        from workloads import make_sym_integrals, orbital_irreps
        orbsym = orbital_irreps(cfg["norb"])
        I = make_sym_integrals(cfg["norb"], cfg["rank"], cfg["seed"], orbsym)
        if not (a.solve_driver or a.kernel_driver):
            print("bench.py: the blocked workloads run under --solve-driver or --kernel-driver "
                  "(the default run reports them in its 'symmetry' section)", file=sys.stderr)
            sys.exit(2)
    else:
        I = make_integrals(cfg["norb"], cfg["rank"], cfg["seed"])

    def context():
        if sym:
            return sb.Context(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, stream=stream,
                              orbsym=orbsym, irrep=cfg["irrep"])
        return sb.Context(cfg["norb"], cfg["na"], cfg["nb"], I.h1, I.eri, stream=stream)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.only_batch:
        print(json.dumps(batch_section(sb, a.precision)))
        return
    if a.only_sym:
        print(json.dumps(sym_section(sb, stream)))
        return
    if a.paper_shapes:
        print(json.dumps(paper_shapes_section(sb, stream, a.precision)))
        return
    if a.solve_driver:
        ctx = context()
        fn = {"sbci1": lambda: ctx.solve(nroots, tol=1e-10, opts=dict(precision="f64"), want_vectors=False),
              "sbci2": lambda: ctx.solve2(nroots, tol=1e-10, want_vectors=False),
              "davidson": lambda: ctx.davidson(nroots, tol=1e-10, want_vectors=False)}[a.solve_driver]
        r = fn()
        torch.cuda.synchronize()
        print(json.dumps({"driver": a.solve_driver, "workload": a.workload, "ndet": ctx.ndet,
                          "nroots": nroots, "energies": [float(e) for e in r.energies],
                          "seconds": r.report["seconds"], "nsigma_f64": r.report["nsigma_f64"]}))
        ctx.close()
        return
    if a.kernel_driver:
        ctx = context()
        c = torch.from_numpy(sigma_inputs(0, 1, ctx.ndet)[0]).cuda()
        if a.kernel_driver != "f64":
            c = c.float()
        out = torch.empty_like(c)
        for _ in range(a.sigma_reps):
            ctx.sigma(c, a.kernel_driver, out=out)
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"driver": a.kernel_driver, "ndet": ctx.ndet, "sigma_calls": a.sigma_reps,
                          "copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}))
        ctx.close()
        return

    # ---- the timed step: one FP64 SBCI1 solve (the paper's form), context
    # build included, to |dE| < 1e-8 Eh for every root
    def step(prec, want_vectors=False):
        ctx = context()
        r = ctx.solve(nroots, tol=1e-10, opts=dict(precision=prec), want_vectors=want_vectors)
        ctx.close()
        return r

    for w in range(a.warmup):
        step("f64")
        note(f"warm-up step {w + 1}/{a.warmup} done")
    torch.cuda.synchronize()
    times, res = [], []
    t0 = time.perf_counter()
    for k in range(a.steps):
        ts = time.perf_counter()
        res.append(step("f64"))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        if (k + 1) % 4 == 0 or k + 1 == a.steps:
            note(f"timed step {k + 1}/{a.steps}: {times[-1]:.3f} s")
    t1 = time.perf_counter()
    ms = (t1 - t0) / a.steps * 1e3
    last = res[-1]
    ctx = context()
    ndet = ctx.ndet
    ctx.close()
    nsig = sum(r.report["nsigma_f64"] for r in res) / a.steps
    value = ndet * nsig / (ms / 1e3) / 1e9

    # ---- outside the timed region: the precision forms (median of 3 solves
    # each, context build included, like the timed step)
    mixed = {}
    for prec in ("bf16", "f32"):
        note(f"precision form {prec}")
        tt, rr = [], None
        for _ in range(3):
            ts = time.perf_counter()
            rr = step(prec)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - ts)
        mixed[prec] = {"time_to_1e8_s": round(statistics.median(tt), 4), "runs": 3,
                       "nsigma": {"f64": rr.report["nsigma_f64"], "low": rr.report["nsigma_low"],
                                  "bf16": rr.report["nsigma_bf16"]},
                       "max_abs_dE_vs_fp64": float(np.abs(np.sort(rr.energies) -
                                                          np.sort(last.energies)).max())}
    t64 = statistics.median(times)

    # ---- sigma per dtype, per kernel (HIP events on the library stream)
    parts = ["same_alpha", "opp_mfma", "transpose", "same_beta", "add_t"]
    sig = {}
    ctx = context()
    c64 = torch.from_numpy(sigma_inputs(0, 1, ndet)[0]).cuda()
    for dt in ["f64", "f32", "bf16"]:
        c = c64 if dt == "f64" else c64.float()
        out, _ = ctx.sigma_timed(c, dt)
        runs = [ctx.sigma_timed(c, dt, out=out)[1] for _ in range(a.sigma_reps)]
        med = np.median(np.array(runs), axis=0)
        sig[dt] = {"gdet_per_s": ndet / (med.sum() / 1e3) / 1e9, "ms": float(med.sum()),
                   "kernels_ms": dict(zip(parts, [round(float(v), 4) for v in med]))}
        del out, c
    # the FP64 sigma with its opposite-spin scatter in FP64 atomics (not
    # reproducible bit for bit) instead of the default fixed point
    ctx.set_deterministic(False)
    out, _ = ctx.sigma_timed(c64, "f64")
    runs = [ctx.sigma_timed(c64, "f64", out=out)[1] for _ in range(a.sigma_reps)]
    med = np.median(np.array(runs), axis=0)
    sig["f64_atomics"] = {"gdet_per_s": ndet / (med.sum() / 1e3) / 1e9, "ms": float(med.sum()),
                          "kernels_ms": dict(zip(parts, [round(float(v), 4) for v in med]))}
    ctx.set_deterministic(True)
    del out
    forms = {"same_spin": ctx.same_form(0), "opposite_spin": ctx.opp_form("f64")}
    del c64
    ctx.close()
    torch.cuda.empty_cache()

    # dominant kernel of the FP64 step: the largest per-kernel share of sigma
    (kname, kdt) = max(((p, "f64") for p in parts), key=lambda k: sig["f64"]["kernels_ms"][k[0]])
    roof = roofline(cfg, ndet, kname, kdt, sig[kdt]["kernels_ms"][kname])
    roof_same = roofline(cfg, ndet, "same_alpha", "f64", sig["f64"]["kernels_ms"]["same_alpha"])

    line = {
        "metric": "sigma=H.c Gdet/s per root; time to |dE|<1e-8 Eh, mixed vs FP64 SBCI",
        "value": round(value, 4),
        "unit": "Gdet/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "norb": cfg["norb"], "nalpha": cfg["na"],
                   "nbeta": cfg["nb"], "ndet": ndet, "nroots": nroots, "eri_rank": cfg["rank"],
                   "seed": cfg["seed"], "step": "context build + FP64 SBCI1 solve to 1e-8 Eh",
                   "parallelism": "1 GPU"},
        "time_to_1e8_s": {"fp64": round(t64, 4), "fp64_runs": a.steps,
                          "fp64_min_max": [round(min(times), 4), round(max(times), 4)],
                          "mixed_bf16": mixed["bf16"]["time_to_1e8_s"],
                          "mixed_f32": mixed["f32"]["time_to_1e8_s"],
                          "speedup_bf16": round(t64 / mixed["bf16"]["time_to_1e8_s"], 3),
                          "speedup_f32": round(t64 / mixed["f32"]["time_to_1e8_s"], 3)},
        "fp64_nsigma": nsig,
        "energies": [float(e) for e in last.energies],
        "mixed": mixed,
        "forms": forms,
        "sigma": sig,
        "roofline": roof,
        "roofline_same": roof_same,
    }
    if a.workload == "cas16" and not a.no_configs:
        note("section cas14")
        line["cas14"] = cas14_section(sb, stream, 3)
    if not a.no_batch:
        note("section batch")
        line["batch"] = batch_section(sb, a.precision)
    if not a.no_configs:
        note("sections cas6, cas10")
        line.update(small_sections(sb, stream))
        if a.workload != "cas16":
            line["cas16"] = cas16_section(sb, stream, a.precision)
        note("section dilute45")
        line["dilute45"] = dilute45_section(sb, stream, a.precision)
        note("section symmetry")
        line["symmetry"] = sym_section(sb, stream)
    if not a.no_cpu_baseline:
        note("cpu baseline and oracle checks")
        xE = None
        if not a.no_configs:
            r = step("f64", want_vectors=True)
            xE = (r.vectors[0], float(r.energies[0]))
        base, checks = oracle_checks(cfg, I, ndet, sb, stream, a.cpu_seconds, xE)
        line["cpu_baseline"] = base
        line["oracle_checks"] = checks
        del xE
    print(json.dumps(line))


if __name__ == "__main__":
    main()
