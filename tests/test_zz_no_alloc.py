"""The allocation-free sigma (sbci_sigma_noalloc) against sbci_sigma, called
through the C ABI: two calls in a row, the second on a smaller input, in
FP64 (1e-12 relative, the sigma parity bar) and FP32 (1e-6 relative), then
the first input again (the shared scratch keeps the last call's contents);
sizes beyond the scratch and the BF16 dtype are refused before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2603_06101_amd as sb  # noqa: E402
from workloads import make_integrals, sigma_inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _noalloc():
    return sb.lib().sbci_sigma_noalloc


def _both(ctx, c, code):
    """(sbci_sigma, sbci_sigma_noalloc) of the same input, both through the C ABI."""
    nvec = c.shape[0]
    ref = torch.empty_like(c)
    got = torch.full_like(c, float("nan"))
    rc = sb.lib().sbci_sigma(ctx.h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                             nvec, code)
    assert rc == 0, sb.lib().sbci_last_error()
    rc = _noalloc()(ctx.h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(got.data_ptr()), nvec, code)
    assert rc == 0, sb.lib().sbci_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy().astype(np.float64), got.cpu().numpy().astype(np.float64)


def _check(ctx, c64, code, tol):
    c = torch.from_numpy(c64).cuda()
    if code == sb.F32:
        c = c.float()
    ref, got = _both(ctx, c, code)
    assert np.all(np.isfinite(got))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= tol, err


def test_noalloc_sigma_matches_sigma_on_two_calls():
    big = make_integrals(10, 20, 0)
    small = make_integrals(8, 16, 1)
    c1 = sb.Context(10, 5, 5, big.h1, big.eri)       # 63,504 determinants, 3 vectors
    c2 = sb.Context(8, 4, 3, small.h1, small.eri)    # 3,920 determinants (Sz != 0), 1 vector
    x1 = sigma_inputs(0, 3, c1.ndet)
    x2 = sigma_inputs(1, 1, c2.ndet)
    print("noalloc: CAS(10,10) nvec 3, then (8,4,3) nvec 1", flush=True)
    for code, tol in ((sb.F64, 1e-12), (sb.F32, 1e-6)):
        _check(c1, x1, code, tol)
        _check(c2, x2, code, tol)
    _check(c1, x1, sb.F64, 1e-12)   # the larger input again after the smaller one
    c1.close()
    c2.close()


def test_noalloc_sigma_refuses_what_it_cannot_hold():
    I = make_integrals(12, 24, 0)
    ctx = sb.Context(12, 6, 6, I.h1, I.eri)          # 853,776 determinants
    nvec = 5                                          # 5 * 853,776 * 8 B > 32 MiB
    c = torch.zeros(nvec * ctx.ndet, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(c)
    rc = _noalloc()(ctx.h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()), nvec, sb.F64)
    assert rc == sb.SBCI_EINVAL and b"64 MiB" in sb.lib().sbci_last_error()
    c32 = torch.zeros(ctx.ndet, dtype=torch.float32, device="cuda")
    o32 = torch.zeros_like(c32)
    rc = _noalloc()(ctx.h, ctypes.c_void_p(c32.data_ptr()), ctypes.c_void_p(o32.data_ptr()), 1, sb.BF16)
    assert rc == sb.SBCI_EINVAL
    # one vector fits: the result equals sbci_sigma's
    x = sigma_inputs(2, 1, ctx.ndet)
    _check(ctx, x, sb.F64, 1e-12)
    ctx.close()
