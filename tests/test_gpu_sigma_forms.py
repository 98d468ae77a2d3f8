"""The forms of sigma against the oracle, through the C ABI: the two
opposite-spin forms (pair and orbital-grouped) and the two same-spin forms
(lists and dense MFMA product).  All compute the Hamiltonian of the Results
section; they differ only in how the work is grouped, so every combination
must match the oracle's sigma."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sigma as OS  # noqa: E402
from workloads import CONFIGS, make_integrals, sigma_inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx(n, na, nb, rank=None, seed=0):
    import paper_2603_06101_amd as sb
    I = make_integrals(n, rank or 2 * n, seed)
    return sb.Context(n, na, nb, I.h1, I.eri), I


# 16-row orbital tiles MT = 1..4, ragged and single-column string groups
# (nq = C(N-1, m_beta-1) = 1, 17, 19, 49, 55), Sz != 0, half filling, a
# fully occupied spin and empty spins
CASES = [(8, 4, 4), (12, 2, 3), (18, 3, 2), (20, 2, 2), (33, 2, 1), (40, 1, 1), (50, 1, 2),
         (9, 4, 5), (5, 5, 5), (7, 0, 3), (6, 3, 0)]


def _forms(ctx, n):
    import paper_2603_06101_amd as sb
    out = ["orbital", "orbital_windowed"]
    try:
        ctx.set_opp_form("pair")
        ctx.opp_form("f64")
        out.append("pair")
    except sb.SbciError:
        assert n >= 40          # the pair form's ERI tile outgrows LDS only there
    return out


@pytest.mark.parametrize("n,na,nb", CASES)
def test_opp_forms_f64_match_oracle(n, na, nb):
    ctx, I = _ctx(n, na, nb, seed=3)
    c = sigma_inputs(5, 2, ctx.ndet)
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    scale = np.abs(want).max()
    for form in _forms(ctx, n):
        ctx.set_opp_form(form)
        if nb > 0 and na > 0:
            assert ctx.opp_form("f64") == form.replace("_windowed", "")
        got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
        err = np.abs(got - want).max() / scale
        assert err <= 1e-12, (form, err)
    ctx.close()


# dense same-spin form: ragged 128-row tiles and K panels (190, 528, 1287,
# 1716 strings), Sz != 0 (different alpha and beta operators), one string
# per spin and empty spins
DENSE_CASES = [(8, 4, 4), (12, 2, 3), (9, 4, 5), (13, 6, 5), (20, 2, 2), (33, 2, 1), (5, 5, 5),
               (7, 0, 3), (6, 3, 0)]


@pytest.mark.parametrize("n,na,nb", DENSE_CASES)
def test_same_dense_f64_matches_oracle(n, na, nb):
    ctx, I = _ctx(n, na, nb, seed=5)
    c = sigma_inputs(7, 2, ctx.ndet)
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    scale = np.abs(want).max()
    ctx.set_same_form("dense")
    assert ctx.same_form(0) == ctx.same_form(1) == "dense"
    for form in _forms(ctx, n):
        ctx.set_opp_form(form)
        got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
        err = np.abs(got - want).max() / scale
        assert err <= 1e-12, (form, err)
    # the lists form on the same context still agrees (dense operators cached)
    ctx.set_same_form("lists")
    ctx.set_opp_form("auto")
    got = ctx.sigma(torch.from_numpy(c).cuda()).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * scale
    ctx.close()


@pytest.mark.parametrize("n,na,nb", [(13, 6, 5), (12, 6, 6), (20, 2, 2), (7, 0, 3), (33, 2, 1)])
def test_same_dense_bf16_error(n, na, nb):
    """BF16 sigma with the dense BF16-MFMA same-spin product (FP32 diagonal in
    the epilogue): error against the FP64 oracle of the order of the BF16
    opposite-spin contraction's, and no worse than twice the lists form's."""
    ctx, I = _ctx(n, na, nb, seed=9)
    c = sigma_inputs(10, 1, ctx.ndet)
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    c32 = torch.from_numpy(c.astype(np.float32)).cuda()
    errs = {}
    for form in ("lists", "dense"):
        ctx.set_same_form(form)
        got = ctx.sigma(c32, dtype="bf16").cpu().numpy()
        errs[form] = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert errs["dense"] < 1e-2, errs
    assert errs["dense"] < 2 * errs["lists"] + 1e-3, errs
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("n,na,nb", [(12, 2, 3), (13, 6, 5), (20, 2, 2)])
def test_same_dense_low_precision(n, na, nb, dtype, tol):
    ctx, I = _ctx(n, na, nb, seed=6)
    c = sigma_inputs(8, 1, ctx.ndet)
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    ctx.set_same_form("dense")
    got = ctx.sigma(torch.from_numpy(c.astype(np.float32)).cuda(), dtype=dtype).cpu().numpy()
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < tol, rel
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("n,na,nb", [(12, 2, 3), (20, 2, 2), (50, 1, 2), (9, 4, 5)])
def test_opp_orbital_low_precision(n, na, nb, dtype, tol):
    ctx, I = _ctx(n, na, nb, seed=4)
    c = sigma_inputs(6, 1, ctx.ndet)
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    for form in ("orbital", "orbital_windowed"):
        ctx.set_opp_form(form)
        got = ctx.sigma(torch.from_numpy(c.astype(np.float32)).cuda(), dtype=dtype).cpu().numpy()
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel < tol, (form, rel)
    ctx.close()


@pytest.mark.parametrize("n,na,nb", [(13, 6, 5), (12, 6, 6), (9, 4, 5), (20, 2, 2), (7, 0, 3)])
def test_bf16_opp_pair_matches_orbital(n, na, nb):
    """The BF16 sigma's two opposite-spin forms multiply the same BF16-rounded
    integrals and coefficients (the pair form gathers from the BF16 copy of C
    that the dense beta product also reads, rows padded to 64) and add the
    products in FP32 MFMAs and FP64 rows, so they agree to accumulation
    rounding, far below the BF16 error; three vectors cover the per-vector
    offsets into the padded copy."""
    ctx, I = _ctx(n, na, nb, seed=2)
    c = sigma_inputs(12, 3, ctx.ndet)
    c32 = torch.from_numpy(c.astype(np.float32)).cuda()
    ctx.set_same_form("dense")
    got = {}
    for form in ("pair", "orbital"):
        ctx.set_opp_form(form)
        got[form] = ctx.sigma(c32, dtype="bf16").cpu().numpy().astype(np.float64)
    for v in range(3):
        a, b = got["pair"][v], got["orbital"][v]
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b), (v, np.linalg.norm(a - b))
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    assert np.linalg.norm(got["pair"] - want) < 2e-2 * np.linalg.norm(want)
    ctx.close()


def test_automatic_form_choice():
    """Near half filling the pair form issues fewer MFMA tiles; with few
    electrons in many orbitals the orbital form does (and at 45 orbitals the
    pair form's ERI tile does not fit in LDS)."""
    ctx, _ = _ctx(14, 7, 7)
    assert all(ctx.opp_form(d) == "pair" for d in ("f64", "f32", "bf16"))
    assert ctx.same_form(0) == ctx.same_form(1) == "lists"
    assert ctx.same_form(0, "f32") == "lists"
    # the BF16 sigma takes the dense BF16-MFMA product from 1024 strings up
    assert ctx.same_form(0, "bf16") == ctx.same_form(1, "bf16") == "dense"
    ctx.close()
    ctx, _ = _ctx(20, 2, 2)
    assert ctx.opp_form("f64") == "orbital"
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_sigma_full_size_dilute45_sampled(dtype):
    """CAS(6e,45o), 201,356,100 determinants (orbital opposite-spin form,
    dense same-spin form): sampled rows
    against the oracle; for FP64 also u.sigma(v) = v.sigma(u)."""
    cfg = CONFIGS["dilute45"]
    n, na, nb = cfg["norb"], cfg["na"], cfg["nb"]
    ctx, I = _ctx(n, na, nb, rank=cfg["rank"], seed=cfg["seed"])
    assert ctx.opp_form(dtype) == "orbital"
    assert ctx.same_form(0) == ctx.same_form(1) == "dense"
    c = sigma_inputs(0, 1, ctx.ndet)[0]
    ct = torch.from_numpy(c if dtype == "f64" else c.astype(np.float32)).cuda()
    s = ctx.sigma(ct, dtype=dtype)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, ctx.ndet - 1], rng.integers(0, ctx.ndet, 200)]))
    want = OS.sigma_rows(n, na, nb, I.h1, I.eri, c, rows)
    got = s.cpu().numpy()[rows].astype(np.float64)
    err = np.abs(got - want).max() / np.abs(want).max()
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-2}[dtype]
    assert err <= tol, err
    if dtype == "f64":
        v = torch.from_numpy(sigma_inputs(1, 1, ctx.ndet)[0]).cuda()
        sv = ctx.sigma(v)
        a, b = float(ct @ sv), float(v @ s)
        assert abs(a - b) <= 1e-10 * max(abs(a), 1.0)
        del v, sv
    del s, ct
    ctx.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sigma_full_size_dilute29_sampled(dtype):
    """CAS(8e,29o), 564,110,001 determinants: a row of sigma (23,751 beta
    strings) exceeds LDS, so the orbital form runs in target windows;
    sampled rows against the oracle."""
    cfg = CONFIGS["dilute29"]
    n, na, nb = cfg["norb"], cfg["na"], cfg["nb"]
    ctx, I = _ctx(n, na, nb, rank=cfg["rank"], seed=cfg["seed"])
    assert ctx.opp_form(dtype) == "orbital"
    c = sigma_inputs(2, 1, ctx.ndet)[0]
    ct = torch.from_numpy(c if dtype == "f64" else c.astype(np.float32)).cuda()
    s = ctx.sigma(ct, dtype=dtype)
    rng = np.random.default_rng(13)
    rows = np.unique(np.concatenate([[0, ctx.ndet - 1], rng.integers(0, ctx.ndet, 150)]))
    want = OS.sigma_rows(n, na, nb, I.h1, I.eri, c, rows)
    got = s.cpu().numpy()[rows].astype(np.float64)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= {"f64": 1e-12, "f32": 1e-5}[dtype], err
    del s, ct
    ctx.close()
    torch.cuda.empty_cache()
