"""Pins of the symmetry-blocked oracle (oracle/symmetry.py) against facts the
mathematics fixes: a totally symmetric Hamiltonian maps each irrep block to
itself, the eight blocks together hold every determinant and every
eigenvalue, and the symmetric integral recipe really is totally symmetric."""
import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import strings as ST
from oracle import symmetry as SY
from workloads import make_sym_integrals, orbital_irreps


CASES = [(6, 3, 3), (6, 2, 3), (7, 3, 2), (8, 4, 4), (5, 1, 0)]


def test_integrals_totally_symmetric():
    n = 9
    o = orbital_irreps(n)
    I = make_sym_integrals(n, 18, 3)
    for p in range(n):
        for q in range(n):
            if o[p] != o[q]:
                assert I.h1[p, q] == 0.0
    g = o[:, None, None, None] ^ o[None, :, None, None] ^ o[None, None, :, None] ^ o[None, None, None, :]
    assert np.all(I.eri[g != 0] == 0.0)
    assert np.abs(I.eri[g == 0]).max() > 1e-3
    assert np.allclose(I.eri, I.eri.transpose(1, 0, 2, 3))
    assert np.allclose(I.eri, I.eri.transpose(2, 3, 0, 1))
    w = np.linalg.eigvalsh(I.eri.reshape(n * n, n * n))
    assert w.min() > -1e-12                     # still positive semidefinite


def test_string_irreps_by_hand():
    o = [0, 1, 2, 3, 4, 5]
    # strings of 2 electrons in 6 orbitals, ascending masks: 0b000011 (orbitals 0,1) first
    g = SY.string_irreps(6, 2, o)
    masks = [int(m) for m in ST.strings(6, 2)]
    assert masks[0] == 0b11 and g[0] == 0 ^ 1
    for m, x in zip(masks, g):
        occ = [p for p in range(6) if (m >> p) & 1]
        assert x == o[occ[0]] ^ o[occ[1]]


@pytest.mark.parametrize("n,na,nb", CASES)
def test_blocks_partition_the_space(n, na, nb):
    o = orbital_irreps(n)
    nfull = len(ST.strings(n, na)) * len(ST.strings(n, nb))
    seen = []
    for g in range(8):
        idx, blocks = SY.block_layout(n, na, nb, o, g)
        assert len(idx) == sum(len(r) * len(c) for _, r, c, _ in blocks)
        for a, rows, cols, off in blocks:
            assert np.all(np.diff(rows) > 0) and np.all(np.diff(cols) > 0)
        seen.append(idx)
    allidx = np.sort(np.concatenate(seen))
    assert np.array_equal(allidx, np.arange(nfull))


@pytest.mark.parametrize("n,na,nb", CASES)
def test_sigma_stays_in_block_and_spectra_add_up(n, na, nb):
    o = orbital_irreps(n)
    I = make_sym_integrals(n, 2 * n, 1)
    Hd = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    full = np.linalg.eigvalsh(Hd)
    parts = []
    rng = np.random.default_rng(5)
    nfull = Hd.shape[0]
    for g in range(8):
        idx, _ = SY.block_layout(n, na, nb, o, g)
        if len(idx) == 0:
            continue
        # H never leaves the block: exact zeros outside it
        c = rng.standard_normal(len(idx))
        s_full = Hd @ SY.embed(c, idx, nfull)
        mask = np.ones(nfull, bool)
        mask[idx] = False
        assert np.all(s_full[mask] == 0.0)
        # the blocked sigma is that restriction, and equals the dense block
        s = SY.sigma(n, na, nb, I.h1, I.eri, o, g, c)
        assert np.abs(s - Hd[np.ix_(idx, idx)] @ c).max() < 1e-12
        parts.append(np.linalg.eigvalsh(Hd[np.ix_(idx, idx)]))
        assert np.abs(SY.hdiag(n, na, nb, I.h1, I.eri, o, g) - np.diag(Hd)[idx]).max() < 1e-12
    assert np.abs(np.sort(np.concatenate(parts)) - full).max() < 1e-10


def test_generic_integrals_do_couple_blocks():
    """The pin above is not vacuous: integrals without the symmetry zeros
    connect the blocks."""
    from workloads import make_integrals
    n, na, nb = 6, 3, 3
    o = orbital_irreps(n)
    I = make_integrals(n, 12, 1)
    Hd = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)
    idx, _ = SY.block_layout(n, na, nb, o, 0)
    mask = np.ones(Hd.shape[0], bool)
    mask[idx] = False
    assert np.abs(Hd[np.ix_(mask, idx)]).max() > 1e-3


@pytest.mark.parametrize("n,na,nb,g", [(6, 3, 3, 0), (7, 3, 2, 5), (8, 4, 4, 3)])
def test_bench_pair_count_matches_tables(n, na, nb, g):
    """The multiply-add count bench.py reports for the blocked opposite-spin
    part equals a count over the oracle's excitation tables: for every
    determinant of the block, the pairs of alpha and beta excitations whose
    classes orbsym[p] ^ orbsym[q] agree."""
    import bench
    o = orbital_irreps(n)
    JA, PA, QA, _ = ST.excitation_table(n, na)
    JB, PB, QB, _ = ST.excitation_table(n, nb)
    idx, _ = SY.block_layout(n, na, nb, o, g)
    nsb = len(ST.strings(n, nb))
    total = 0
    for d in idx:
        ia, ib = divmod(int(d), nsb)
        ca = np.bincount([o[p] ^ o[q] for p, q in zip(PA[ia], QA[ia])], minlength=8)
        cb = np.bincount([o[p] ^ o[q] for p, q in zip(PB[ib], QB[ib])], minlength=8)
        total += int(ca @ cb)
    assert bench.sym_pair_count(n, na, nb, o, g) == total
