"""Point-group symmetry blocking of the determinant space (oracle; test
infrastructure, used only by the tests, the smoke check and the benchmark's
CPU baseline).

The paper solves each molecule inside one irreducible representation of its
point group (the IRep column of the Section S3.1 table; the determinant
counts printed there are the full C(norb, na) * C(norb, nb) products, not
the size of one irrep's block).  With an abelian group whose irreps
are labelled 0..7 and multiply by XOR (D2h and its subgroups):

* orbital p carries the irrep orbsym[p];
* a string's irrep is the XOR of the irreps of its occupied orbitals;
* determinant |Ia, Ib> has irrep irr(Ia) XOR irr(Ib);
* the integrals are totally symmetric: h_pq = 0 unless orbsym[p] ==
  orbsym[q], and (pq|rs) = 0 unless orbsym[p] ^ orbsym[q] ^ orbsym[r] ^
  orbsym[s] == 0, so H couples only determinants of one irrep and the
  determinants of irrep G span an invariant subspace.

Block layout of a vector of irrep G (the layout the HIP library uses; stated
here, in the oracle, independently of it): for a = 0..7, block a holds the
determinants whose alpha string has irrep a and whose beta string has irrep
a ^ G, as a row-major matrix [alpha strings of irrep a, ascending mask]
x [beta strings of irrep a ^ G, ascending mask]; the blocks follow one
another in order of a.

sigma on the block is the definition itself: embed the blocked vector in the
full space (zeros elsewhere), apply the full-space sigma of ``oracle.sigma``
and keep the block's entries.  Pins (tests/test_oracle_symmetry.py): the full
sigma of an embedded vector is exactly zero outside the block; the spectra of
the eight blocked Hamiltonians together are the full spectrum; block sizes
add up to the full determinant count.
"""
from __future__ import annotations

import numpy as np

from . import sigma as _sg
from . import strings as _st


def string_irreps(norb: int, nelec: int, orbsym) -> np.ndarray:
    """Irrep of every string (ascending mask order): XOR over occupied orbitals."""
    out = []
    for m in _st.strings(norb, nelec):
        m = int(m)
        g = 0
        for p in range(norb):
            if (m >> p) & 1:
                g ^= int(orbsym[p])
        out.append(g)
    return np.array(out, dtype=np.int64)


def block_layout(norb: int, na: int, nb: int, orbsym, irrep: int):
    """Blocks of the irrep-``irrep`` determinant space.

    Returns (index, blocks): index[d] is the full-space determinant index
    Ia * Nb + Ib of blocked position d; blocks is a list of (a, alpha string
    indices, beta string indices, offset) for a = 0..7.
    """
    ia = string_irreps(norb, na, orbsym)
    ib = string_irreps(norb, nb, orbsym)
    nsb = len(ib)
    index, blocks, off = [], [], 0
    for a in range(8):
        rows = np.nonzero(ia == a)[0]
        cols = np.nonzero(ib == (a ^ irrep))[0]
        blocks.append((a, rows, cols, off))
        for r in rows:
            index.extend(int(r) * nsb + cols)
        off += len(rows) * len(cols)
    return np.array(index, dtype=np.int64), blocks


def embed(c_blocked: np.ndarray, index: np.ndarray, ndet_full: int) -> np.ndarray:
    c = np.asarray(c_blocked, dtype=np.float64)
    out = np.zeros(c.shape[:-1] + (ndet_full,))
    out[..., index] = c
    return out


def sigma(norb, na, nb, h1, eri, orbsym, irrep, c_blocked):
    """sigma = H c on the irrep block: full-space sigma of the embedded vector,
    restricted to the block."""
    index, _ = block_layout(norb, na, nb, orbsym, irrep)
    nfull = len(_st.strings(norb, na)) * len(_st.strings(norb, nb))
    full = _sg.sigma(norb, na, nb, h1, eri, embed(c_blocked, index, nfull))
    return full[..., index]


def hdiag(norb, na, nb, h1, eri, orbsym, irrep):
    """Diagonal of H on the block (the full-space diagonal, restricted)."""
    index, _ = block_layout(norb, na, nb, orbsym, irrep)
    nfull = len(_st.strings(norb, na)) * len(_st.strings(norb, nb))
    return _sg.hdiag(norb, na, nb, h1, eri, nfull)[index]


class Operator:
    """Blocked H as a callable on [nvec, ndet_block] arrays (plus its diagonal)."""

    def __init__(self, norb, na, nb, h1, eri, orbsym, irrep):
        self.args = (norb, na, nb, h1, eri)
        self.orbsym, self.irrep = list(orbsym), int(irrep)
        self.index, self.blocks = block_layout(norb, na, nb, orbsym, irrep)
        self.ndet = len(self.index)
        self.nfull = len(_st.strings(norb, na)) * len(_st.strings(norb, nb))

    def __call__(self, c):
        full = _sg.sigma(*self.args, embed(c, self.index, self.nfull))
        return full[..., self.index]

    def diag(self):
        return _sg.hdiag(*self.args, self.nfull)[self.index]
