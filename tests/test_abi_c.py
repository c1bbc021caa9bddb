"""The C ABI from plain C: tests/abi_c/abi_check.c, compiled by gcc against
include/rhmc.h and librhmc.so with HIP device buffers (no Python or torch
in the program).

* CPU: the header is valid C11 and the program links against the library;
  without a GPU every call returns an error status (nothing aborts).
* GPU: a point source on unit links gives exactly +-1/2 at the eight
  neighbours (Eq. stag), and a MIXED multi-shift solve meets its FP64
  residual, all through the C entry points.
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1106_5673_amd")


def _compile(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "librhmc.so")):
        pytest.skip("librhmc.so is not built")
    exe = str(tmp_path / "abi_check")
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-O2", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", f"-I{ROOT}/include", os.path.join(ROOT, "tests", "abi_c", "abi_check.c"),
           f"-L{LIBDIR}", "-lrhmc", "-L/opt/rocm/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{LIBDIR}", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_program_compiles_and_links(tmp_path):
    _compile(tmp_path)


@pytest.mark.gpu
def test_c_program_runs_on_gpu(tmp_path):
    exe = _compile(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "abi ok" in r.stdout
