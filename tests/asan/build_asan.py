"""Build the host-sanitizer check: libsbci with its host code under
AddressSanitizer (device code unchanged), and host_driver linked to it.
Outputs next to this file: _build/ (objects), libsbci_asan.so, host_driver.

Usage: python tests/asan/build_asan.py   (also run by __graft_entry__.build)
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2603_06101_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/bin/amdclang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-Wno-unused-value"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed:\n{r.stderr[-3000:]}")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def comp(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        _run([HIPCC, *FLAGS, *SAN, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    lib = os.path.join(HERE, "libsbci_asan.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs])
    drv_o = os.path.join(BUILD, "host_driver.o")
    _run([CLANG, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *SAN[:2],
          "-Wno-unused-result", "-Wno-unused-value", "-I" + os.path.join(ROOT, "include"),
          os.path.join(HERE, "host_driver.cpp"), "-c", "-o", drv_o])
    exe = os.path.join(HERE, "host_driver")
    # host-only link: the sanitizer runtime goes into the executable
    link = [CLANG, "-fsanitize=address", drv_o, "-o", exe, "-L" + HERE, "-lsbci_asan",
            "-Wl,-rpath,$ORIGIN", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    _run(link)
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    build(verbose=True)
