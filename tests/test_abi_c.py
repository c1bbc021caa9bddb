"""The C ABI from plain C: tests/abi_c/abi_check.c, compiled by gcc against
include/rhmc.h and librhmc.so with HIP device buffers (no Python or torch
in the program).

* CPU: the header is valid C11 and the program links against the library;
  without a GPU every call returns an error status (nothing aborts).
* CPU: every public struct has the layout of its ctypes mirror.
* GPU: a point source on unit links gives exactly +-1/2 at the eight
  neighbours (Eq. stag), and a MIXED multi-shift solve meets its FP64
  residual, all through the C entry points.
"""

import ctypes
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


def test_struct_layouts_match_binding(tmp_path):
    """Every public struct has the same size and field offsets in C (gcc,
    tests/abi_c/layout.c) as its ctypes mirror in the Python binding, and the
    two declare the same fields."""
    import re

    from paper_1106_5673_amd import rhmc

    exe = str(tmp_path / "layout")
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{ROOT}/include", os.path.join(ROOT, "tests", "abi_c", "layout.c"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes, offsets = {}, {}
    for line in filter(None, out):
        name, value = line.split()
        if "." in name:
            offsets[name] = int(value)
        else:
            sizes[name] = int(value)
    # every typedef'd struct of the header is covered by layout.c
    header = open(os.path.join(ROOT, "include", "rhmc.h")).read()
    declared = set(re.findall(r"^\}\s*(rhmc_\w+);", header, re.M)) - {"rhmc_status", "rhmc_mode"}
    assert declared == set(sizes)
    for name, size in sizes.items():
        cls = getattr(rhmc, name)
        assert ctypes.sizeof(cls) == size, name
        fields = [f[0] for f in cls._fields_]
        c_fields = [k.split(".", 1)[1] for k in offsets if k.startswith(name + ".")]
        # the binding renames C's `lambda` (a Python keyword) to `lambda_`
        assert [f.rstrip("_") for f in fields] == c_fields, name
        for f in fields:
            assert getattr(cls, f).offset == offsets[f"{name}.{f.rstrip('_')}"], (name, f)
