"""CPU-side checks of libsbci.so: it loads, exports every entry point of
include/sbci.h, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2603_06101_amd as sb
from workloads import make_integrals

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sbci.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sbci_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(sb.LIB_PATH):
        pytest.fail("libsbci.so not built (run __graft_entry__.build())")
    L = sb.lib()
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    # the binding covers the same set
    assert sorted(n for n, _, _ in sb.SIGNATURES) == names


def test_default_opts_are_the_papers_thresholds():
    o = sb.default_opts()
    assert (o.eps0, o.r0, o.b_th, o.eps1, o.x_th1, o.x_th2, o.r1, o.max_cycle) == \
        (1e-10, 1e-5, 1e-2, 1e-7, 0.1, 1.2, 1.0, 20)


def _create(n, na, nb, h, g):
    out = ctypes.c_void_p()
    rc = sb.lib().sbci_create(n, na, nb, h.ctypes.data, g.ctypes.data, ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("n,na,nb", [(0, 0, 0), (64, 1, 1), (4, 5, 1), (4, 1, -1)])
def test_create_rejects_bad_sizes(n, na, nb):
    h = np.zeros((4, 4))
    g = np.zeros((4,) * 4)
    rc, out = _create(n, na, nb, h, g)
    assert rc == sb.SBCI_EINVAL and not out.value
    assert sb.lib().sbci_last_error()


def test_create_rejects_unsymmetric_integrals():
    I = make_integrals(4, 8, 0)
    h = I.h1.copy()
    h[0, 1] += 1e-6
    rc, _ = _create(4, 2, 2, h, I.eri)
    assert rc == sb.SBCI_EINVAL and b"symmetric" in sb.lib().sbci_last_error()
    g = I.eri.copy()
    g[0, 1, 2, 3] += 1e-6
    rc, _ = _create(4, 2, 2, I.h1, g)
    assert rc == sb.SBCI_EINVAL
    g = I.eri.copy()
    g[0, 0, 0, 0] = np.nan
    rc, _ = _create(4, 2, 2, I.h1, g)
    assert rc == sb.SBCI_EINVAL


def test_null_context_calls_fail_cleanly():
    L = sb.lib()
    assert L.sbci_sigma(None, None, None, 1, 0) == sb.SBCI_EINVAL
    assert L.sbci_step(None, None, None) == sb.SBCI_EINVAL
    assert L.sbci_ndet(None) == -1
    assert L.sbci_destroy(None) == sb.SBCI_OK


def test_symmetry_entry_points_reject_null_arguments():
    I = make_integrals(4, 8, 0)
    out = ctypes.c_void_p()
    rc = sb.lib().sbci_create_sym(4, 2, 2, I.h1.ctypes.data, I.eri.ctypes.data, None, 0,
                                  ctypes.byref(out))
    assert rc == sb.SBCI_EINVAL and not out.value and b"orbsym" in sb.lib().sbci_last_error()
    blocks = np.zeros(24, dtype=np.int64)
    assert sb.lib().sbci_sym_blocks(None, blocks.ctypes.data) == sb.SBCI_EINVAL


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the structure of the same name in sbci.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("sbci_opts", sb.Opts), ("sbci_report", sb.Report), ("sbci_step_info", sb.StepInfo),
             ("sbci_batch_config", sb.BatchConfig), ("sbci_batch_inst", sb.BatchInst),
             ("sbci_batch_report", sb.BatchReport)]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sbci.h"', "int main(void) {"]
    want = []
    for cname, py in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(py))
        for f in py._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f[0]}));')
            want.append(getattr(py, f[0]).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want
