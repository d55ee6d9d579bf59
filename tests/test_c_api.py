"""The C ABI from a plain C program (tests/c_api_demo.c), no Python in the process: built with gcc
against include/tpcf.h and the in-tree libtpcf.so. On the CPU it runs the argument and state
checks that need no device; on the GPU it computes zeta for a seeded catalogue, compared with the
oracle at the FP64 bar."""
import os
import subprocess

import numpy as np
import pytest

import catalogs
import oracle
import paper_2604_08855_amd as tpcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def demo(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("capi") / "c_api_demo")
    libdir = os.path.dirname(tpcf.library_path())
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c_api_demo.c"), "-L", libdir, "-ltpcf",
                           "-Wl,-rpath," + libdir, "-o", exe])
    return exe


def test_c_program_validates_arguments(demo):
    out = subprocess.run([demo, "validate"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "validate: ok" in out.stdout


@pytest.mark.gpu
def test_c_program_computes_zeta(demo, tmp_path):
    cat = catalogs.uniform(4000, 100.0, 401)
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([cat.n], dtype=np.int64).tofile(f)
        np.concatenate([cat.x, cat.y, cat.z]).astype(np.float64).tofile(f)
    out = subprocess.run([demo, "compute", str(inp), str(outp)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    z = np.fromfile(outp, dtype=np.float64).reshape(5, 8, 8)
    ref = oracle.zeta(cat.x, cat.y, cat.z, None, 100.0, True, 8, 4.0, 30.0, 4)
    assert f"{ref.npairs} pairs" in out.stdout
    for l in range(5):
        assert np.abs(z[l] - ref.zeta[l]).max() <= 1e-10 * np.abs(ref.zeta[l]).max()
