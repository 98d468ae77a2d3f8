"""Python binding of libsbci.so (argument marshalling only).

Every step of the sigma build and of the SBCI1 / Davidson solvers runs in the
HIP library; this module only converts arguments.  PyTorch supplies device
memory (tensors on ``cuda``) and the stream.  There is no CPU fallback: if
the library is missing the import of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbci.so")

SBCI_OK, SBCI_EINVAL, SBCI_ENOMEM, SBCI_EDEVICE, SBCI_ENOCONV, SBCI_ENUMERIC = 0, -1, -2, -3, -4, -5
F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
OPP_FORMS = {"auto": 0, "pair": 1, "orbital": 2, "orbital_windowed": 3, "class_mfma": 4}
SAME_FORMS = {"auto": 0, "lists": 1, "dense": 2}
REASONS = {0: "", 1: "converged", 2: "S62a", 3: "S62b", 4: "S62c", 5: "max_cycle", 6: "rank",
           7: "coef", 8: "refine", 9: "handover_k"}


class SbciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sbci error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [
        ("eps0", ctypes.c_double), ("r0", ctypes.c_double),
        ("b_th", ctypes.c_double), ("eps1", ctypes.c_double),
        ("x_th1", ctypes.c_double), ("x_th2", ctypes.c_double),
        ("r1", ctypes.c_double),
        ("max_cycle", ctypes.c_int), ("max_steps", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("mix_eps0", ctypes.c_double), ("mix_r0", ctypes.c_double),
        ("mix_stall", ctypes.c_int),
        ("precond_floor", ctypes.c_double), ("lindep", ctypes.c_double),
        ("max_space", ctypes.c_int),
        ("x0", ctypes.POINTER(ctypes.c_double)),
        ("bf16_eps0", ctypes.c_double), ("bf16_r0", ctypes.c_double),
        ("max_cycle2", ctypes.c_int), ("s78_printed", ctypes.c_int),
        ("nconv0", ctypes.c_int),
        ("xc0", ctypes.POINTER(ctypes.c_double)), ("ec0", ctypes.POINTER(ctypes.c_double)),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("nroots_converged", ctypes.c_int), ("nsteps", ctypes.c_int), ("nrestarts", ctypes.c_int),
        ("nsigma_f64", ctypes.c_int64), ("nsigma_low", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("t_converged", ctypes.c_double * 16), ("resid", ctypes.c_double * 16),
        ("peak_vector_bytes", ctypes.c_int64), ("nsigma_bf16", ctypes.c_int64),
    ]


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("root", ctypes.c_int), ("segment", ctypes.c_int), ("t", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("E", ctypes.c_double), ("dE", ctypes.c_double), ("dz", ctypes.c_double),
        ("b", ctypes.c_double), ("c", ctypes.c_double), ("k", ctypes.c_double),
        ("xnorm", ctypes.c_double), ("seconds", ctypes.c_double),
        ("reason", ctypes.c_int),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["reason"] = REASONS.get(self.reason, str(self.reason))
        return d


_lib = None

# (name, restype, argtypes) of every entry point declared in include/sbci.h
_P, _D, _I, _I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64


class BatchConfig(ctypes.Structure):
    _fields_ = [("threads", _I), ("wg_per_cu", _I), ("order", _I), ("k_panel", _I), ("max_team", _I),
                ("team_wait_us", _I), ("queue_reserve", _I)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchInst(ctypes.Structure):
    _fields_ = [
        ("status", _I), ("nroots_converged", _I), ("nsteps", _I), ("nrestarts", _I),
        ("nsigma_f64", _I), ("nsigma_low", _I), ("t_start", _D), ("t_end", _D),
        ("resid", _D * 4), ("t_same", _D), ("t_opp", _D),
    ]


class BatchReport(ctypes.Structure):
    _fields_ = [
        ("seconds", _D), ("span_seconds", _D), ("nsigma_f64", _I64), ("nsigma_low", _I64), ("det_sigma", _I64),
        ("nsteps", _I64), ("nrestarts", _I64), ("ninst_converged", _I),
        ("threads", _I), ("wg_per_cu", _I), ("order", _I), ("k_panel", _I), ("max_team", _I),
        ("team_wait_us", _I), ("nteams", _I), ("team_workgroups", _I), ("team_timeouts", _I),
        ("queue_reserve", _I),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(StepInfo), ctypes.c_void_p)

SIGNATURES = [
    ("sbci_default_opts", None, [ctypes.POINTER(Opts)]),
    ("sbci_last_error", ctypes.c_char_p, []),
    ("sbci_create", _I, [_I, _I, _I, _P, _P, ctypes.POINTER(_P)]),
    ("sbci_create_sym", _I, [_I, _I, _I, _P, _P, _P, _I, ctypes.POINTER(_P)]),
    ("sbci_sym_blocks", _I, [_P, _P]),
    ("sbci_destroy", _I, [_P]),
    ("sbci_set_stream", _I, [_P, _P]),
    ("sbci_ndet", _I64, [_P]),
    ("sbci_nstrings", _I64, [_P, _I]),
    ("sbci_tables", _I, [_P, _I, _P, ctypes.POINTER(_I64)]),
    ("sbci_hdiag", _I, [_P, _P]),
    ("sbci_sigma", _I, [_P, _P, _P, _I, _I]),
    ("sbci_sigma_noalloc", _I, [_P, _P, _P, _I, _I]),
    ("sbci_sigma_timed", _I, [_P, _P, _P, _I, _I, ctypes.POINTER(ctypes.c_float)]),
    ("sbci_set_deterministic", _I, [_P, _I]),
    ("sbci_set_opp_form", _I, [_P, _I]),
    ("sbci_get_opp_form", _I, [_P, _I, ctypes.POINTER(_I)]),
    ("sbci_set_same_form", _I, [_P, _I]),
    ("sbci_set_progress", _I, [_P, PROGRESS_FN, _P]),
    ("sbci_get_same_form", _I, [_P, _I, _I, ctypes.POINTER(_I)]),
    ("sbci_solve", _I, [_P, _I, _D, ctypes.POINTER(Opts), _P, _P, ctypes.POINTER(Report)]),
    ("sbci_begin", _I, [_P, _I, _D, ctypes.POINTER(Opts)]),
    ("sbci_step", _I, [_P, ctypes.POINTER(StepInfo), ctypes.POINTER(_I)]),
    ("sbci_finish", _I, [_P, _P, _P, ctypes.POINTER(Report)]),
    ("sbci_iterate", _I, [_P, _P]),
    ("sbci_set_trace", _I, [_P, _I]),
    ("sbci_trace", _I, [_P, ctypes.POINTER(StepInfo), _I]),
    ("sbci_davidson", _I, [_P, _I, _D, ctypes.POINTER(Opts), _P, _P, ctypes.POINTER(Report)]),
    ("sbci_solve2", _I, [_P, _I, _D, ctypes.POINTER(Opts), _P, _P, ctypes.POINTER(Report)]),
    ("sbci_batch_create", _I, [_I, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    ("sbci_batch_destroy", _I, [_P]),
    ("sbci_batch_ndet", _I64, [_P, _I]),
    ("sbci_batch_solve", _I, [_P, _P, _D, ctypes.POINTER(Opts), ctypes.POINTER(BatchConfig), _P,
                              ctypes.POINTER(BatchInst), ctypes.POINTER(BatchReport)]),
    ("sbci_batch_tune", _I, [_P, _P, _D, ctypes.POINTER(Opts), ctypes.POINTER(BatchConfig), _P,
                             ctypes.POINTER(BatchConfig), ctypes.POINTER(_I)]),
    ("sbci_batch_vectors", _I, [_P, _I, _P]),
]


def lib():
    """Load libsbci.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_06101_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != SBCI_OK and rc not in allow:
        raise SbciError(rc, lib().sbci_last_error().decode())
    return rc


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().sbci_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = DTYPES[v]
        setattr(o, k, v)
    return o


def _torch():
    import torch
    return torch


@dataclass
class SolveResult:
    energies: np.ndarray
    vectors: object          # torch tensor [nroots, ndet] float64 on cuda, or None
    report: dict
    trace: list
    status: int


class Context:
    """One FCI problem (norb, nalpha, nbeta, h1, eri) resident on the GPU.

    With orbsym (irrep label 0..7 per orbital) the context holds only the
    determinants of irreducible representation ``irrep`` (sbci_create_sym):
    vectors are in its block layout and ``ndet`` is the blocked count."""

    def __init__(self, norb, nalpha, nbeta, h1, eri, stream=None, orbsym=None, irrep=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libsbci needs a HIP device")
        self.norb, self.na, self.nb = norb, nalpha, nbeta
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        self._keep = (h1, eri)
        h = _P()
        if orbsym is None:
            _check(lib().sbci_create(norb, nalpha, nbeta, h1.ctypes.data, eri.ctypes.data,
                                     ctypes.byref(h)))
        else:
            os_ = np.ascontiguousarray(orbsym, dtype=np.int32)
            if os_.shape != (norb,):
                raise ValueError("orbsym must have norb entries")
            _check(lib().sbci_create_sym(norb, nalpha, nbeta, h1.ctypes.data, eri.ctypes.data,
                                         os_.ctypes.data, int(irrep), ctypes.byref(h)))
        self.symmetric = orbsym is not None
        self.h = h
        self.ndet = lib().sbci_ndet(h)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().sbci_set_stream(h, ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().sbci_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sym_blocks(self):
        """(alpha rows, beta columns, offsets) of the eight irrep blocks."""
        out = np.zeros(24, dtype=np.int64)
        _check(lib().sbci_sym_blocks(self.h, out.ctypes.data))
        return out[:8].copy(), out[8:16].copy(), out[16:].copy()

    def nstrings(self, spin):
        return lib().sbci_nstrings(self.h, spin)

    def tables(self, which):
        """which: 0/1 alpha/beta strings (uint64 as int64), 2/3 excitation tables (raw bytes)."""
        torch = _torch()
        nb = _I64()
        _check(lib().sbci_tables(self.h, which, None, ctypes.byref(nb)))
        if which in (0, 1):
            out = torch.empty(nb.value // 8, dtype=torch.int64, device="cuda")
        else:
            out = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        if nb.value:
            _check(lib().sbci_tables(self.h, which, ctypes.c_void_p(out.data_ptr()), None))
        return out

    def hdiag(self):
        torch = _torch()
        out = torch.empty(self.ndet, dtype=torch.float64, device="cuda")
        _check(lib().sbci_hdiag(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def sigma(self, c, dtype="f64", out=None):
        """sigma = H c for c [nvec, ndet] (or [ndet]) on cuda; float64 for f64, float32 otherwise."""
        torch = _torch()
        code = DTYPES[dtype] if isinstance(dtype, str) else dtype
        want = torch.float64 if code == F64 else torch.float32
        if c.dtype != want or not c.is_cuda or not c.is_contiguous():
            raise ValueError(f"c must be a contiguous cuda {want} tensor")
        nvec = 1 if c.dim() == 1 else c.shape[0]
        if c.numel() != nvec * self.ndet:
            raise ValueError("c has the wrong size")
        if out is None:
            out = torch.empty_like(c)
        _check(lib().sbci_sigma(self.h, ctypes.c_void_p(c.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), nvec, code))
        return out

    def set_deterministic(self, on=True):
        """FP64 sigma the same to the last bit on every call (default) or, off, FP64 atomics."""
        _check(lib().sbci_set_deterministic(self.h, 1 if on else 0))

    def set_opp_form(self, form):
        """Force the opposite-spin form ("auto", "pair", "orbital", "orbital_windowed";
        "class_mfma" on symmetry-blocked contexts) of later sigma calls."""
        _check(lib().sbci_set_opp_form(self.h, OPP_FORMS[form]))

    def opp_form(self, dtype="f64"):
        """The opposite-spin form ("pair" or "orbital") sigma calls of this dtype use."""
        f = _I(0)
        _check(lib().sbci_get_opp_form(self.h, DTYPES[dtype], ctypes.byref(f)))
        return {1: "pair", 2: "orbital"}[f.value]

    def set_progress(self, fn):
        """Call fn(step: dict) after every solver step (None removes it).  fn runs on
        the calling thread, inside the solve."""
        if fn is None:
            self._progress = None
            _check(lib().sbci_set_progress(self.h, PROGRESS_FN(), None))
            return
        def tramp(info, _user):
            fn(info.contents.as_dict())
        self._progress = PROGRESS_FN(tramp)   # kept alive while set
        _check(lib().sbci_set_progress(self.h, self._progress, None))

    def set_same_form(self, form):
        """Force the same-spin form ("auto", "lists" or "dense") of later sigma calls."""
        _check(lib().sbci_set_same_form(self.h, SAME_FORMS[form]))

    def same_form(self, spin=0, dtype="f64"):
        """The same-spin form ("lists" or "dense") sigma calls of this dtype use for spin 0 or 1."""
        f = _I(0)
        _check(lib().sbci_get_same_form(self.h, spin, DTYPES[dtype], ctypes.byref(f)))
        return {v: k for k, v in SAME_FORMS.items()}[f.value]

    def sigma_timed(self, c, dtype="f64", out=None):
        """sigma with per-kernel HIP-event timings: (out, [alpha, opp, transpose, beta, add] ms)."""
        torch = _torch()
        code = DTYPES[dtype] if isinstance(dtype, str) else dtype
        nvec = 1 if c.dim() == 1 else c.shape[0]
        if out is None:
            out = torch.empty_like(c)
        ms = (ctypes.c_float * 5)()
        _check(lib().sbci_sigma_timed(self.h, ctypes.c_void_p(c.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), nvec, code, ms))
        return out, [float(v) for v in ms]

    def _run(self, fn, nroots, tol, opts, want_vectors):
        torch = _torch()
        o = opts if isinstance(opts, Opts) else default_opts(**(opts or {}))
        e = np.zeros(nroots)
        vec = torch.empty((nroots, self.ndet), dtype=torch.float64, device="cuda") \
            if want_vectors else None
        rep = Report()
        rc = fn(self.h, nroots, tol, ctypes.byref(o), e.ctypes.data,
                ctypes.c_void_p(vec.data_ptr()) if vec is not None else None, ctypes.byref(rep))
        _check(rc, allow=(SBCI_ENOCONV,))
        return SolveResult(e, vec, _report_dict(rep, nroots), self.trace(), rc)

    @staticmethod
    def _resume(o, xc, ec):
        """Point opts at converged roots xc [k, N_det] (numpy or a torch tensor,
        copied to the host) and energies ec [k] (or None); returns the host
        arrays, which must outlive the call."""
        if xc is None:
            return ()
        if hasattr(xc, "detach"):
            xc = xc.detach().to("cpu").numpy()
        xc = np.ascontiguousarray(np.atleast_2d(xc), dtype=np.float64)
        o.nconv0 = xc.shape[0]
        o.xc0 = xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if ec is not None:
            ec = np.ascontiguousarray(ec, dtype=np.float64)
            if ec.shape != (xc.shape[0],):
                raise ValueError("ec must hold one energy per row of xc")
            o.ec0 = ec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return (xc, ec)

    def solve(self, nroots, tol=1e-10, opts=None, want_vectors=True, x0=None, xc=None, ec=None):
        """SBCI1 for the lowest nroots states; x0: optional host start vector (numpy).
        xc / ec: resume after len(xc) converged roots (their vectors and, optionally,
        energies); the result holds all nroots roots."""
        o = opts if isinstance(opts, Opts) else default_opts(**(opts or {}))
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64)
            o.x0 = x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep = self._resume(o, xc, ec)  # noqa: F841 (kept alive across the call)
        return self._run(lib().sbci_solve, nroots, tol, o, want_vectors)

    def davidson(self, nroots, tol=1e-10, opts=None, want_vectors=True):
        return self._run(lib().sbci_davidson, nroots, tol, opts, want_vectors)

    def solve2(self, nroots, tol=1e-10, opts=None, want_vectors=True):
        """SBCI2 (pairs of states; FP64) for the lowest nroots states."""
        return self._run(lib().sbci_solve2, nroots, tol, opts, want_vectors)

    def begin(self, nroots, tol=1e-10, opts=None, x0=None, xc=None, ec=None):
        o = opts if isinstance(opts, Opts) else default_opts(**(opts or {}))
        if x0 is not None:
            self._x0 = np.ascontiguousarray(x0, dtype=np.float64)
            o.x0 = self._x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._resume_keep = self._resume(o, xc, ec)
        self._opts = o
        _check(lib().sbci_begin(self.h, nroots, tol, ctypes.byref(o)))
        self._nroots = nroots

    def step(self):
        info = StepInfo()
        done = _I(0)
        _check(lib().sbci_step(self.h, ctypes.byref(info), ctypes.byref(done)))
        return info.as_dict(), bool(done.value)

    def finish(self, want_vectors=True):
        torch = _torch()
        e = np.zeros(self._nroots)
        vec = torch.empty((self._nroots, self.ndet), dtype=torch.float64, device="cuda") \
            if want_vectors else None
        rep = Report()
        rc = lib().sbci_finish(self.h, e.ctypes.data,
                               ctypes.c_void_p(vec.data_ptr()) if vec is not None else None,
                               ctypes.byref(rep))
        _check(rc, allow=(SBCI_ENOCONV,))
        return SolveResult(e, vec, _report_dict(rep, self._nroots), self.trace(), rc)

    def iterate(self):
        """Current iterate x of the root being solved (FP64, unnormalised) on cuda."""
        torch = _torch()
        x = torch.empty(self.ndet, dtype=torch.float64, device="cuda")
        _check(lib().sbci_iterate(self.h, ctypes.c_void_p(x.data_ptr())))
        return x

    def trace(self):
        n = lib().sbci_trace(self.h, None, 0)
        if n <= 0:
            return []
        buf = (StepInfo * n)()
        m = lib().sbci_trace(self.h, buf, n)
        return [buf[i].as_dict() for i in range(m)]


@dataclass
class BatchResult:
    energies: list           # per instance: numpy array of its roots' energies
    status: np.ndarray       # per-instance sbci_status
    report: dict
    rc: int
    instances: list          # per-instance dicts: nsteps, times, residuals, ...


class Batch:
    """Many independent instances solved by SBCI1 in one persistent-kernel graph launch.

    instances: sequence of (norb, nalpha, nbeta, h1, eri) with host numpy integrals.
    """

    def __init__(self, instances):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libsbci needs a HIP device")
        n = len(instances)
        norb = np.array([t[0] for t in instances], dtype=np.int32)
        na = np.array([t[1] for t in instances], dtype=np.int32)
        nb = np.array([t[2] for t in instances], dtype=np.int32)
        self._ints = [(np.ascontiguousarray(t[3], dtype=np.float64),
                       np.ascontiguousarray(t[4], dtype=np.float64)) for t in instances]
        hp = (ctypes.c_void_p * n)(*[h.ctypes.data for h, _ in self._ints])
        ep = (ctypes.c_void_p * n)(*[e.ctypes.data for _, e in self._ints])
        h = _P()
        _check(lib().sbci_batch_create(n, norb.ctypes.data, na.ctypes.data, nb.ctypes.data,
                                       ctypes.cast(hp, _P), ctypes.cast(ep, _P), ctypes.byref(h)))
        self.h = h
        self.n = n
        self.ndet = [lib().sbci_batch_ndet(h, i) for i in range(n)]
        self._nroots = None

    def close(self):
        if getattr(self, "h", None):
            lib().sbci_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _roots(nroots, n):
        r = np.full(n, nroots, dtype=np.int32) if np.isscalar(nroots) else \
            np.ascontiguousarray(nroots, dtype=np.int32)
        if r.shape != (n,):
            raise ValueError("nroots must be a scalar or one entry per instance")
        return r

    def solve(self, nroots, tol=1e-10, opts=None, config=None):
        r = self._roots(nroots, self.n)
        o = opts if isinstance(opts, Opts) else default_opts(**(opts or {}))
        e = np.full(int(r.sum()), np.nan)
        info = (BatchInst * self.n)()
        rep = BatchReport()
        cfg = None
        if config is not None:
            cfg = config if isinstance(config, BatchConfig) else BatchConfig(**config)
        rc = lib().sbci_batch_solve(self.h, r.ctypes.data, tol, ctypes.byref(o),
                                    ctypes.byref(cfg) if cfg is not None else None,
                                    e.ctypes.data, info, ctypes.byref(rep))
        # SBCI_EDEVICE with team timeouts counted: per-instance outcomes, outputs written
        _check(rc, allow=(SBCI_ENOCONV, SBCI_ENUMERIC) + ((SBCI_EDEVICE,) if rep.team_timeouts > 0 else ()))
        self._nroots = r
        parts = np.split(e, np.cumsum(r)[:-1])
        inst = []
        for i in range(self.n):
            q = info[i]
            d = {f: getattr(q, f) for f, _ in BatchInst._fields_ if f != "resid"}
            d["resid"] = list(q.resid[:int(r[i])])
            inst.append(d)
        st = np.array([d["status"] for d in inst], dtype=np.int32)
        return BatchResult(parts, st, rep.as_dict(), rc, inst)

    def tune(self, nroots, tol=1e-10, opts=None):
        """Run the autotuner; returns (best config dict, [(config dict, ms), ...])."""
        r = self._roots(nroots, self.n)
        o = opts if isinstance(opts, Opts) else default_opts(**(opts or {}))
        best = BatchConfig()
        cap = 32
        ms = np.zeros(cap)
        cand = (BatchConfig * cap)()
        nc = _I(cap)
        _check(lib().sbci_batch_tune(self.h, r.ctypes.data, tol, ctypes.byref(o), ctypes.byref(best),
                                     ms.ctypes.data, cand, ctypes.byref(nc)))
        k = min(nc.value, cap)
        return best.as_dict(), [(cand[i].as_dict(), float(ms[i])) for i in range(k)]

    def vectors(self, inst):
        """Converged FP64 vectors of instance inst from the last solve: [nconv, ndet] on cuda."""
        torch = _torch()
        k = int(self._nroots[inst])
        out = torch.full((k, self.ndet[inst]), float("nan"), dtype=torch.float64, device="cuda")
        _check(lib().sbci_batch_vectors(self.h, inst, ctypes.c_void_p(out.data_ptr())))
        return out


def _report_dict(rep: Report, nroots: int) -> dict:
    k = min(nroots, 16)
    return dict(nroots_converged=rep.nroots_converged, nsteps=rep.nsteps, nrestarts=rep.nrestarts,
                nsigma_f64=rep.nsigma_f64, nsigma_low=rep.nsigma_low, seconds=rep.seconds,
                t_converged=list(rep.t_converged[:k]), resid=list(rep.resid[:k]),
                peak_vector_bytes=rep.peak_vector_bytes, nsigma_bf16=rep.nsigma_bf16)


def decode_table(raw, nstr, s):
    """Split the raw 8-byte excitation records into (J, p, q, sign) numpy arrays [nstr, s]."""
    a = np.asarray(raw.cpu().numpy() if hasattr(raw, "cpu") else raw, dtype=np.uint8)
    rec = a.view(np.dtype([("J", "<i4"), ("p", "u1"), ("q", "u1"), ("sign", "i1"), ("pad", "u1")]))
    rec = rec.reshape(nstr, s) if s else rec.reshape(nstr, 0)
    return rec
