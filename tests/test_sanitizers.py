"""Host sanitizers (CPU only): the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
runs its pins, and the library's host side (argument checks, state handling, buffer bookkeeping of
the C ABI) built with the same sanitizers runs the argument-validation checks from plain C and from
Python. Any report fails the test (UBSan halts on the first error; leak checks are off, as the
Python interpreter and the HIP runtime keep allocations alive until exit).

Device code is never built with a sanitizer here: only host objects are instrumented (hipcc takes
each sanitizer flag behind -Xarch_host).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "tpcf_oracle.c")
CSRC = os.path.join(ROOT, "paper_2604_08855_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2604_08855_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _clean(out: str):
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehavior"):
        assert marker not in out, out[-4000:]


def _gcc_runtime(name: str) -> str:
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def test_oracle_pins_under_asan_ubsan(tmp_path):
    """Every oracle pin (tests/test_oracle_pins.py) and the cheap pins of the mutation test, with
    the oracle built -fsanitize=address,undefined."""
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preloaded library is already present; the sanitizer runtime must come first")
    so = str(tmp_path / "libtpcf_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", so, ORACLE_SRC,
                           "-lm"])
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=_gcc_runtime("libasan.so"), TPCF_ORACLE_LIB=so,
               OMP_NUM_THREADS="4")
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                          "tests/test_oracle_pins.py",
                          "tests/test_oracle_mutations.py::test_unmutated_oracle_passes_cheap_pins"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    text = out.stdout + out.stderr
    _clean(text)
    assert out.returncode == 0, text[-4000:]
    assert " passed" in out.stdout


def test_abi_validation_under_asan_ubsan(tmp_path):
    """The C ABI's host code (api.hip) built with -fsanitize=address,undefined for the host pass
    only, linked with the device objects of the regular build: the plain C program's validation
    steps and the Python ABI checks (tests/test_abi_cpu.py) run clean."""
    objs = [os.path.join(BUILD, f + ".o") for f in ("grid", "sweep", "edge", "pivots")]
    if not all(os.path.exists(o) for o in objs) or not os.path.exists(CLANG):
        pytest.skip("library objects not built (python paper_2604_08855_amd/build.py) or no clang")
    res = subprocess.check_output([CLANG, "-print-resource-dir"], text=True).strip()
    found = [os.path.join(r, f) for r, _, fs in os.walk(os.path.join(res, "lib")) for f in fs
             if f in ("libclang_rt.asan-x86_64.so", "libclang_rt.asan.so")]
    if not found:
        pytest.skip("no clang AddressSanitizer runtime")
    rt = found[0]
    rt_dir = os.path.dirname(rt)
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preloaded library is already present; the sanitizer runtime must come first")
    d = str(tmp_path)
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    api_o = os.path.join(d, "api_san.o")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, "api.hip"),
                           "-o", api_o], stderr=subprocess.DEVNULL)
    lib = os.path.join(d, "libtpcf.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address,undefined", "-shared-libsan", "-o", lib, api_o, *objs])
    demo = os.path.join(d, "c_api_demo")
    subprocess.check_call([CLANG, "-std=c11", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-shared-libsan", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c_api_demo.c"), "-L" + d, "-ltpcf", "-Wl,-rpath," + d,
                           "-Wl,-rpath," + rt_dir, "-o", demo])
    env = dict(os.environ, **SAN_ENV)
    out = subprocess.run([demo, "validate"], env=env, capture_output=True, text=True, timeout=300)
    _clean(out.stdout + out.stderr)
    assert out.returncode == 0 and "validate: ok" in out.stdout, out.stdout + out.stderr
    env_py = dict(env, LD_PRELOAD=rt, TPCF_LIBRARY_PATH=lib)
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                          "tests/test_abi_cpu.py"], cwd=ROOT, env=env_py, capture_output=True, text=True,
                         timeout=600)
    text = out.stdout + out.stderr
    _clean(text)
    assert out.returncode == 0, text[-4000:]
    assert " passed" in out.stdout
