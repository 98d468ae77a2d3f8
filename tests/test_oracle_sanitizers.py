"""The oracle's C string sigma under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only): a small driver compiled with the sanitizers runs
oracle_sigma, oracle_sigma_rows and oracle_hdiag on edge-case shapes (an
empty spin, a full spin, Sz != 0, one orbital) and must finish with no report;
its sigma must equal the regular build's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sigma as OS
from workloads import make_integrals

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")

SRC = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "csrc", "sigma_ref.c")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include "SRCFILE"
static void *rd(FILE *f, size_t n) { void *p = malloc(n ? n : 1); if (fread(p, 1, n, f) != n) exit(3); return p; }
int main(int argc, char **argv) {
  FILE *f = fopen(argv[1], "rb");
  int hdr[3];
  if (fread(hdr, sizeof(int), 3, f) != 3) return 3;
  const int n = hdr[0], na = hdr[1], nb = hdr[2];
  int64_t nd, nr;
  if (fread(&nd, 8, 1, f) != 1 || fread(&nr, 8, 1, f) != 1) return 3;
  double *h1 = rd(f, sizeof(double) * n * n), *eri = rd(f, sizeof(double) * n * n * n * n);
  double *c = rd(f, sizeof(double) * nd);
  int64_t *rows = rd(f, sizeof(int64_t) * nr);
  fclose(f);
  double *s = malloc(sizeof(double) * nd), *d = malloc(sizeof(double) * nd), *sr = malloc(sizeof(double) * (nr ? nr : 1));
  int rc = oracle_sigma(n, na, nb, h1, eri, c, s);
  rc |= oracle_hdiag(n, na, nb, h1, eri, d);
  rc |= oracle_sigma_rows(n, na, nb, h1, eri, c, rows, nr, sr);
  FILE *o = fopen(argv[2], "wb");
  fwrite(s, sizeof(double), nd, o); fwrite(d, sizeof(double), nd, o); fwrite(sr, sizeof(double), nr, o);
  fclose(o);
  free(h1); free(eri); free(c); free(rows); free(s); free(d); free(sr);
  return rc;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    src = d / "driver.c"
    src.write_text(DRIVER.replace("SRCFILE", SRC))
    exe = d / "driver"
    r = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", str(src), "-o", str(exe), "-lm"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    return exe, d


@pytest.mark.parametrize("n,na,nb", [(1, 1, 0), (4, 2, 2), (5, 0, 2), (6, 6, 3), (7, 3, 4), (8, 4, 4)])
def test_oracle_sigma_clean_under_asan_ubsan(driver, n, na, nb):
    from math import comb
    exe, d = driver
    I = make_integrals(n, 2 * n, n + na)
    nd = comb(n, na) * comb(n, nb)
    c = np.random.default_rng(n).standard_normal(nd)
    rows = np.unique(np.random.default_rng(1).integers(0, nd, min(nd, 7))).astype(np.int64)
    fin, fout = d / f"in_{n}_{na}_{nb}.bin", d / f"out_{n}_{na}_{nb}.bin"
    with open(fin, "wb") as f:
        f.write(np.array([n, na, nb], dtype=np.int32).tobytes())
        f.write(np.array([nd, rows.size], dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(I.h1, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(I.eri, dtype=np.float64).tobytes())
        f.write(c.tobytes())
        f.write(rows.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), str(fin), str(fout)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    out = np.fromfile(fout, dtype=np.float64)
    s, dg, sr = out[:nd], out[nd:2 * nd], out[2 * nd:]
    want = OS.sigma(n, na, nb, I.h1, I.eri, c)
    assert np.abs(s - want).max() <= 1e-13 * max(1.0, np.abs(want).max())
    assert np.abs(sr - want[rows]).max() <= 1e-13 * max(1.0, np.abs(want).max())
    assert np.abs(dg - OS.hdiag(n, na, nb, I.h1, I.eri, nd)).max() <= 1e-13 * max(1.0, np.abs(dg).max())
