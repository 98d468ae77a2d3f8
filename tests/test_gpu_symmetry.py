"""Point-group blocked contexts (sbci_create_sym) against the symmetry-blocked
oracle: block layout, diagonal, sigma in FP64, FP32 and BF16 (the
opposite-spin part on MFMA, and in the vector pair form), and the solvers'
energies against the spectrum of the blocked Hamiltonian."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import hamiltonian as H  # noqa: E402
from oracle import sigma as OS  # noqa: E402
from oracle import symmetry as SY  # noqa: E402
from workloads import CONFIGS, make_integrals, make_sym_integrals, orbital_irreps, sigma_inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx(n, na, nb, irrep, orbsym=None, seed=0):
    import paper_2603_06101_amd as sb
    o = orbital_irreps(n) if orbsym is None else np.asarray(orbsym)
    I = make_sym_integrals(n, 2 * n, seed, o)
    return sb.Context(n, na, nb, I.h1, I.eri, orbsym=o, irrep=irrep), I, o


# half filling, Sz != 0, an empty spin, a fully occupied spin, labels that
# leave irreps unused, and more than 8 orbitals (labels repeat)
CASES = [
    (6, 3, 3, None), (7, 3, 2, None), (8, 4, 4, None), (9, 4, 5, None), (5, 0, 2, None),
    (6, 6, 3, None), (8, 3, 3, [0, 0, 1, 1, 2, 3, 3, 0]), (12, 2, 3, None), (11, 5, 5, None),
]


def _irreps_with_dets(n, na, nb, o):
    out = []
    for g in range(8):
        idx, _ = SY.block_layout(n, na, nb, o, g)
        if len(idx):
            out.append(g)
    return out


@pytest.mark.parametrize("n,na,nb,orbsym", CASES)
def test_layout_diag_and_sigma_f64(n, na, nb, orbsym):
    o = orbital_irreps(n) if orbsym is None else np.asarray(orbsym)
    for g in _irreps_with_dets(n, na, nb, o):
        ctx, I, o = _ctx(n, na, nb, g, orbsym, seed=g)
        idx, blocks = SY.block_layout(n, na, nb, o, g)
        assert ctx.ndet == len(idx)
        rows, cols, offs = ctx.sym_blocks()
        for a, r, c, off in blocks:
            assert (rows[a], cols[a], offs[a]) == (len(r), len(c), off)
        d = ctx.hdiag().cpu().numpy()
        assert np.abs(d - SY.hdiag(n, na, nb, I.h1, I.eri, o, g)).max() < 1e-12
        c = sigma_inputs(g, 3, ctx.ndet)
        want = SY.sigma(n, na, nb, I.h1, I.eri, o, g, c)
        got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-12 * scale, (g, np.abs(got - want).max() / scale)
        c32 = torch.from_numpy(c.astype(np.float32)).cuda()
        got32 = ctx.sigma(c32, dtype="f32").cpu().numpy()
        rel = np.linalg.norm(got32 - want) / np.linalg.norm(want)
        assert rel < 2e-6, (g, rel)
        # BF16 operands in the opposite-spin MFMA (8-bit mantissa), FP32 elsewhere
        gotb = ctx.sigma(c32, dtype="bf16").cpu().numpy()
        relb = np.linalg.norm(gotb - want) / np.linalg.norm(want)
        assert relb < 1e-2, (g, relb)
        # the class MFMA form in FP64 and FP32 (the default there is the vector form)
        ctx.set_opp_form("class_mfma")
        gotm = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
        assert np.abs(gotm - want).max() <= 1e-12 * scale, (g, np.abs(gotm - want).max() / scale)
        gotm32 = ctx.sigma(c32, dtype="f32").cpu().numpy()
        assert np.linalg.norm(gotm32 - want) / np.linalg.norm(want) < 2e-6
        gotmb = ctx.sigma(c32, dtype="bf16").cpu().numpy()
        assert np.array_equal(gotmb, gotb) or np.linalg.norm(gotmb - gotb) / np.linalg.norm(want) < 1e-6
        ctx.close()


@pytest.mark.parametrize("g", [0, 5])
def test_sigma_with_integral_rows_beyond_lds(g):
    """30 orbitals, 2 + 2 electrons: the workgroup's integral rows (58 x 465 in
    FP64, 216 KB) exceed the LDS budget, so the contraction reads them from
    global memory instead of staging them."""
    n, na, nb = 30, 2, 2
    ctx, I, o = _ctx(n, na, nb, g, seed=4)
    c = sigma_inputs(1, 2, ctx.ndet)
    want = SY.sigma(n, na, nb, I.h1, I.eri, o, g, c)
    got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    got32 = ctx.sigma(torch.from_numpy(c.astype(np.float32)).cuda(), dtype="f32").cpu().numpy()
    assert np.linalg.norm(got32 - want) / np.linalg.norm(want) < 2e-6
    ctx.close()


def test_bad_forms_and_arguments_are_refused():
    import paper_2603_06101_amd as sb
    ctx, I, o = _ctx(6, 3, 3, 0)
    c = torch.zeros(ctx.ndet, dtype=torch.float32, device="cuda")
    ctx.set_opp_form("pair")
    with pytest.raises(sb.SbciError):
        ctx.sigma(c, dtype="bf16")       # the vector pair form has no BF16 flavour
    with pytest.raises(sb.SbciError):
        ctx.set_opp_form("orbital")      # no orbital form on blocked contexts
    ctx.close()
    # integrals that break the symmetry
    J = make_integrals(6, 12, 0)
    with pytest.raises(sb.SbciError):
        sb.Context(6, 3, 3, J.h1, J.eri, orbsym=orbital_irreps(6), irrep=0)
    # an irrep that no determinant has: 2 orbitals of irreps 0 and 1
    K = make_sym_integrals(2, 4, 0, [0, 1])
    with pytest.raises(sb.SbciError):
        sb.Context(2, 1, 1, K.h1, K.eri, orbsym=[0, 1], irrep=2)
    with pytest.raises(sb.SbciError):
        sb.Context(2, 1, 1, K.h1, K.eri, orbsym=[0, 9], irrep=0)
    # an unblocked context has no blocks and no class MFMA form
    U = sb.Context(6, 3, 3, J.h1, J.eri)
    with pytest.raises(sb.SbciError):
        U.sym_blocks()
    with pytest.raises(sb.SbciError):
        U.set_opp_form("class_mfma")
    U.close()


@pytest.mark.parametrize("form", ["auto", "class_mfma"])
@pytest.mark.parametrize("n,na,nb,g", [(8, 4, 4, 0), (9, 4, 5, 3), (7, 3, 2, 1), (12, 2, 3, 6)])
def test_blocked_sigma_f64_bitwise_reproducible(n, na, nb, g, form):
    """The blocked FP64 sigma is the same to the last bit from call to call:
    its opposite-spin scatter (pair and MFMA forms) accumulates in 64-bit
    fixed point, the other parts sum in a fixed order.  Calls of another size
    in between change how the waves interleave; the FP64-atomic scatter
    (reproducibility off) meets the same parity bar."""
    ctx, I, o = _ctx(n, na, nb, g, seed=g)
    ctx.set_opp_form(form)
    c = torch.from_numpy(sigma_inputs(g, 2, ctx.ndet)).cuda()
    want = SY.sigma(n, na, nb, I.h1, I.eri, o, g, c.cpu().numpy())
    scale = np.abs(want).max()
    ref = ctx.sigma(c).clone()
    assert np.abs(ref.cpu().numpy() - want).max() <= 1e-12 * scale
    for _ in range(4):
        ctx.sigma(c[:1].contiguous())
        got = ctx.sigma(c)
        assert torch.equal(got.view(torch.int64), ref.view(torch.int64))
    ctx.set_deterministic(False)
    r = ctx.sigma(c).cpu().numpy()
    assert np.abs(r - want).max() <= 1e-12 * scale
    ctx.close()


@pytest.mark.parametrize("det", [True, False])
@pytest.mark.parametrize("form", ["auto", "class_mfma"])
def test_blocked_sigma_f64_carries_a_nan(det, form):
    """A NaN in c reaches sigma (the solvers stop on non-finite reductions):
    the NaN's own entry is NaN, and every entry that stays finite equals the
    oracle's.  The fixed-point scatter turns every row that gathers the NaN's
    row into NaN; the FP64 atomics only the entries it reaches."""
    n, na, nb, g = 8, 4, 4, 0
    ctx, I, o = _ctx(n, na, nb, g, seed=1)
    ctx.set_deterministic(det)
    ctx.set_opp_form(form)
    c = sigma_inputs(1, 1, ctx.ndet)
    c[0, 11] = np.nan
    want = SY.sigma(n, na, nb, I.h1, I.eri, o, g, c)
    got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    assert np.isnan(got[0, 11])
    both = np.isfinite(got) & np.isfinite(want)
    assert both.sum() > 0
    assert np.abs(got[both] - want[both]).max() <= 1e-12 * np.abs(want[both]).max()
    ctx.close()


def test_class_of_more_than_64_pairs_uses_the_vector_form():
    """Labels that put 12 of 13 orbitals in irrep 0 make pair class 0 hold 79
    pairs (more than an MFMA class tile takes): FP64 still runs (the vector
    pair form); the MFMA form, and with it BF16, is refused."""
    import paper_2603_06101_amd as sb
    o = [0] * 12 + [3]
    ctx, I, _ = _ctx(13, 3, 2, 0, orbsym=o, seed=2)
    c = sigma_inputs(5, 1, ctx.ndet)[0]
    idx, _ = SY.block_layout(13, 3, 2, np.asarray(o), 0)
    want = SY.sigma(13, 3, 2, I.h1, I.eri, np.asarray(o), 0, c[None])[0]
    got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    with pytest.raises(sb.SbciError):
        ctx.sigma(torch.from_numpy(c.astype(np.float32)).cuda(), dtype="bf16")
    ctx.set_opp_form("class_mfma")
    with pytest.raises(sb.SbciError):
        ctx.sigma(torch.from_numpy(c).cuda())
    ctx.close()


@pytest.mark.parametrize("n,na,nb,g", [(8, 4, 4, 0), (8, 4, 4, 5), (7, 3, 4, 2), (9, 4, 4, 1)])
def test_solvers_reach_the_blocked_spectrum(n, na, nb, g):
    ctx, I, o = _ctx(n, na, nb, g, seed=11)
    idx, _ = SY.block_layout(n, na, nb, o, g)
    Hd = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)[np.ix_(idx, idx)]
    w = np.linalg.eigvalsh(Hd)
    nroots = 3
    r1 = ctx.solve(nroots, tol=1e-10)
    assert r1.status == 0
    assert np.abs(np.sort(r1.energies) - w[:nroots]).max() < 1e-8, (r1.energies, w[:nroots])
    X = r1.vectors.cpu().numpy()
    assert np.abs(X @ X.T - np.eye(nroots)).max() < 1e-8
    r2 = ctx.solve2(nroots, tol=1e-10)
    assert np.abs(np.sort(r2.energies) - w[:nroots]).max() < 1e-8
    rd = ctx.davidson(nroots, tol=1e-10)
    assert np.abs(np.sort(rd.energies) - w[:nroots]).max() < 1e-8
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("n,na,nb,g", [(8, 4, 4, 0), (8, 4, 4, 5), (7, 3, 4, 2), (9, 4, 4, 1)])
def test_precision_forms_reach_the_blocked_spectrum(n, na, nb, g, prec):
    """The FP32 and BF16 precision forms (low-precision sigma and FP32
    vectors, FP64 reductions and refinement) on few-hundred-determinant
    blocks whose lowest states lie
    within about 5e-5 Eh of single diagonal entries.  (7,3,4, irrep 2) and
    (8,4,4, irrep 5) once stopped with a non-finite reduction: a step whose
    new iterate has norm |k| << 1 amplified the FP32 images' error until the
    iterate overflowed; such a step now hands over to FP64 before it is
    taken."""
    ctx, I, o = _ctx(n, na, nb, g, seed=11)
    idx, _ = SY.block_layout(n, na, nb, o, g)
    Hd = H.dense_h_slater_condon(n, na, nb, I.h1, I.eri)[np.ix_(idx, idx)]
    w = np.linalg.eigvalsh(Hd)
    nroots = 3
    rm = ctx.solve(nroots, tol=1e-10, opts=dict(precision=prec))
    assert rm.status == 0
    assert np.abs(np.sort(rm.energies) - w[:nroots]).max() < 1e-8, (rm.energies, w[:nroots])
    ctx.close()


def test_full_size_cas14_sym_sampled_and_solved():
    """CAS(14e,14o), orbital irreps p mod 8, irrep 0: 1,472,928 determinants.
    Sampled rows of the blocked sigma against the oracle's rows of the full
    sigma of the embedded vector; then five roots whose energies are Rayleigh
    quotients of orthonormal vectors with converged residuals, the same in the
    FP32 precision form and in SBCI2."""
    cfg = CONFIGS["cas14_sym"]
    n, na, nb, g = cfg["norb"], cfg["na"], cfg["nb"], cfg["irrep"]
    ctx, I, o = _ctx(n, na, nb, g, seed=cfg["seed"])
    assert ctx.ndet == 1472928
    idx, _ = SY.block_layout(n, na, nb, o, g)
    c = sigma_inputs(3, 1, ctx.ndet)[0]
    got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    full = SY.embed(c, idx, 3432 * 3432)
    rng = np.random.default_rng(0)
    sample = np.concatenate([rng.choice(ctx.ndet, 300, replace=False), [0, ctx.ndet - 1]])
    want = OS.sigma_rows(n, na, nb, I.h1, I.eri, full, idx[sample])
    assert np.abs(got[sample] - want).max() <= 1e-12 * np.abs(want).max()
    r = ctx.solve(5, tol=1e-10)
    assert r.status == 0
    X = r.vectors
    S = ctx.sigma(X)
    rq = (X * S).sum(1).cpu().numpy()
    res = torch.linalg.norm(S - torch.tensor(rq, device=X.device)[:, None] * X, dim=1).cpu().numpy()
    assert np.abs(rq - r.energies).max() < 1e-9
    assert res.max() < 3e-5
    assert np.abs((X @ X.T).cpu().numpy() - np.eye(5)).max() < 1e-8
    for prec in ("f32", "bf16"):
        rm = ctx.solve(5, tol=1e-10, opts=dict(precision=prec), want_vectors=False)
        assert rm.status == 0, prec
        assert np.abs(np.sort(rm.energies) - np.sort(r.energies)).max() < 1e-8, prec
    r2 = ctx.solve2(5, tol=1e-10, want_vectors=False)
    assert np.abs(np.sort(r2.energies) - np.sort(r.energies)).max() < 1e-8
    ctx.close()
