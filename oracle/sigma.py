"""sigma = H c in the string basis (oracle), via the plain C routine.

``csrc/sigma_ref.c`` evaluates each determinant row from the Slater-Condon
rules (see its header).  It is compiled with gcc by ``build()`` (called from
``__graft_entry__.build``) into ``oracle/liboracle_sigma.so``; nothing of the
HIP library is involved.  Pins: equality with the two dense builders of
``hamiltonian`` on every size they reach, linearity, symmetry, transpose
symmetry, and closed forms (tests/test_oracle_hamiltonian.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "sigma_ref.c")
_LIB = os.path.join(_HERE, "liboracle_sigma.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_sigma.argtypes = [ctypes.c_int] * 3 + [dp] * 4
        lib.oracle_sigma_rows.argtypes = [ctypes.c_int] * 3 + [dp] * 3 + [i64p, ctypes.c_int64, dp]
        lib.oracle_hdiag.argtypes = [ctypes.c_int] * 3 + [dp] * 3
        for f in (lib.oracle_sigma, lib.oracle_sigma_rows, lib.oracle_hdiag):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sigma(norb, na, nb, h1, eri, c):
    """sigma = H c for one vector or a stack [nvec, ndet]; FP64."""
    lib = _load()
    h1 = np.ascontiguousarray(h1, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    single = c.ndim == 1
    cs = np.atleast_2d(c)
    out = np.empty_like(cs)
    for i in range(cs.shape[0]):
        ci = np.ascontiguousarray(cs[i])
        oi = np.empty_like(ci)
        rc = lib.oracle_sigma(norb, na, nb, _dp(h1), _dp(eri), _dp(ci), _dp(oi))
        if rc:
            raise ValueError("oracle_sigma rejected its arguments")
        out[i] = oi
    return out[0] if single else out


def sigma_rows(norb, na, nb, h1, eri, c, rows):
    """sigma[rows] only (for sampled checks at sizes where a full sigma is too slow)."""
    lib = _load()
    h1 = np.ascontiguousarray(h1, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(len(rows))
    rc = lib.oracle_sigma_rows(norb, na, nb, _dp(h1), _dp(eri), _dp(c),
                               rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               len(rows), _dp(out))
    if rc:
        raise ValueError("oracle_sigma_rows rejected its arguments")
    return out


def hdiag(norb, na, nb, h1, eri, ndet):
    lib = _load()
    h1 = np.ascontiguousarray(h1, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    out = np.empty(ndet)
    rc = lib.oracle_hdiag(norb, na, nb, _dp(h1), _dp(eri), _dp(out))
    if rc:
        raise ValueError("oracle_hdiag rejected its arguments")
    return out


class Operator:
    """Matrix-free H for the eigensolver references (wraps ``sigma``)."""

    def __init__(self, norb, na, nb, h1, eri):
        from math import comb
        self.norb, self.na, self.nb = norb, na, nb
        self.h1 = np.ascontiguousarray(h1, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.ndet = comb(norb, na) * comb(norb, nb)
        self.nsigma = 0

    def __call__(self, c):
        c = np.asarray(c)
        self.nsigma += 1 if c.ndim == 1 else c.shape[0]
        return sigma(self.norb, self.na, self.nb, self.h1, self.eri, c)

    def diag(self):
        return hdiag(self.norb, self.na, self.nb, self.h1, self.eri, self.ndet)
