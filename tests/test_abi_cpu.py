"""C-ABI checks that need no GPU: the library loads, exports every declared function, and every
argument error that the host can detect comes back as the documented status code without a
device call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2604_08855_amd as tpcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpcf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpcf_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(tpcf.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.check_output(["nm", "-D", "--defined-only", tpcf.library_path()]).decode()
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [f for f in declared_functions() if f not in names]
    assert not missing, missing
    assert sorted(tpcf.exported_symbols()) == declared_functions()
    assert "gfx950" in tpcf.version()


def _ctx():
    return tpcf.Context(device=0, stream=None)


def _code(fn, *a, **k):
    with pytest.raises(tpcf.TpcfError) as e:
        fn(*a, **k)
    return e.value.code


def test_set_bins_validation():
    c = _ctx()
    assert _code(c.set_bins, 0, 1.0, 2.0, 2) == 1
    assert _code(c.set_bins, 33, 1.0, 2.0, 2) == 1
    assert _code(c.set_bins, 4, -1.0, 2.0, 2) == 1
    assert _code(c.set_bins, 4, 2.0, 2.0, 2) == 1
    assert _code(c.set_bins, 4, 1.0, float("nan"), 2) == 1
    assert _code(c.set_bins, 4, 1.0, float("inf"), 2) == 1
    assert _code(c.set_bins, 4, 1.0, 2.0, -1) == 1
    assert _code(c.set_bins, 4, 1.0, 2.0, 11) == 1
    c.set_bins(4, 0.0, 2.0, 10)  # valid: rmin = 0, lmax = 10, nbins = 32 below
    c.set_bins(32, 1.0, 2.0, 0)


def test_precision_and_tuning_validation():
    c = _ctx()
    assert _code(c.set_precision, 7) == 1
    c.set_precision("mixed")
    c.set_precision("fp64")
    assert _code(c.set_tuning, -1.0, 0, 0) == 1
    assert _code(c.set_tuning, 0.0, -2, 0) == 1
    assert _code(c.set_tuning, 0.0, 0, 100) == 1  # not a multiple of 64
    c.set_tuning(20.0, 4, 256)
    assert _code(c.degenerate) == 2  # no bins, no catalogue
    lib = ctypes.CDLL(tpcf.library_path())
    cb = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)(lambda p, u: None)
    lib.tpcf_set_allocator.argtypes = [ctypes.c_void_p] * 4
    assert lib.tpcf_set_allocator(c._h, None, ctypes.cast(cb, ctypes.c_void_p), None) == 1
    assert lib.tpcf_set_allocator(c._h, None, None, None) == 0
    assert _code(c.set_phase_aligned, 2) == 1
    assert _code(c.set_phase_aligned, -2) == 1
    for mode in (-1, 0, 1):
        c.set_phase_aligned(mode)


def test_autotune_validation_on_host():
    c = _ctx()
    assert _code(c.autotune, 1.5) == 1
    assert _code(c.autotune, -0.1) == 1
    assert _code(c.autotune, float("nan")) == 1
    assert _code(c.autotune) == 2  # no bins
    c.set_bins(4, 1.0, 10.0, 2)
    assert _code(c.autotune, 0.5) == 2  # no catalogue
    assert "catalogue" in tpcf._lib.tpcf_last_error(c._h).decode()


def test_edge_correct_validation_on_host():
    c = _ctx()
    a = np.zeros((3, 2, 2))
    p = a.ctypes.data_as(ctypes.c_void_p)
    assert tpcf._lib.tpcf_edge_correct(c._h, 0, p, p, p, 0) == 1
    assert tpcf._lib.tpcf_edge_correct(c._h, 1, None, p, p, 0) == 1
    assert tpcf._lib.tpcf_edge_correct(c._h, 1, p, p, p, 7) == 1
    assert tpcf._lib.tpcf_edge_correct(c._h, 1, p, p, p, 0) == 2  # bins not set


def test_compute_before_setup_is_a_state_error():
    c = _ctx()
    out = np.zeros(1)
    rc = tpcf._lib.tpcf_compute_zeta(c._h, out.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == 2
    assert "set_bins" in tpcf._lib.tpcf_last_error(c._h).decode()
    c.set_bins(4, 1.0, 10.0, 2)
    rc = tpcf._lib.tpcf_compute_zeta(c._h, out.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == 2
    rc = tpcf._lib.tpcf_compute_zeta_range(c._h, 0, 1, out.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == 2
    rc = tpcf._lib.tpcf_debug_pair_counts(c._h, out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 2
    rc = tpcf._lib.tpcf_pair_sums(c._h, 1, None, out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 2


def test_catalog_validation_on_host():
    c = _ctx()
    c.set_bins(4, 1.0, 10.0, 2)
    x = np.array([1.0, 2.0, 3.0])
    assert _code(c.set_catalog, x, x, x, box=0.0) == 1
    assert _code(c.set_catalog, x, x, x, box=float("inf")) == 1
    assert _code(c.set_catalog, np.array([1.0, np.nan, 2.0]), x, x, box=50.0) == 1
    assert _code(c.set_catalog, x, x, x, np.array([1.0, np.inf, 1.0]), box=50.0) == 1
    # periodic needs rmax < box/2
    assert _code(c.set_catalog, x, x, x, box=19.0, periodic=True) == 1
    # non-periodic points must lie in [0, box)
    assert _code(c.set_catalog, np.array([1.0, 2.0, 50.0]), x, x, box=50.0, periodic=False) == 1
    assert _code(c.set_catalog, np.array([1.0, -1e-9, 3.0]), x, x, box=50.0, periodic=False) == 1
    assert _code(c.set_catalog, np.array([1e9, 2.0, 3.0]), x, x, box=50.0, periodic=True) == 1
    assert _code(c.set_catalog, np.array([1.0, np.nan, 2.0]), x, x, box=50.0) == 1
    assert "non-finite" in tpcf._lib.tpcf_last_error(c._h).decode()
    # raw ABI: negative n and NULL arrays
    rc = tpcf._lib.tpcf_set_catalog(c._h, -1, None, None, None, None, 50.0, 1, 0)
    assert rc == 1
    rc = tpcf._lib.tpcf_set_catalog(c._h, 3, None, None, None, None, 50.0, 1, 0)
    assert rc == 1
    rc = tpcf._lib.tpcf_set_catalog(c._h, 3, None, None, None, None, 50.0, 1, 9)
    assert rc == 1


def test_batch_validation_on_host():
    c = _ctx()
    c.set_bins(4, 1.0, 10.0, 2)
    x = np.arange(6, dtype=np.float64)
    with pytest.raises(tpcf.TpcfError) as e:
        c.compute_batch([0, 4, 3], x, x, x, None, 50.0, True)
    assert e.value.code == 1
    with pytest.raises(tpcf.TpcfError) as e:
        c.compute_batch([1, 3, 6], x, x, x, None, 50.0, True)
    assert e.value.code == 1
    with pytest.raises(tpcf.TpcfError) as e:
        c.compute_batch([0, 3, 6], x, x, x, None, [50.0, 15.0], True)  # second box too small
    assert e.value.code == 1


def test_null_context_is_rejected():
    assert tpcf._lib.tpcf_set_bins(None, 4, 1.0, 2.0, 2) == 1
    assert tpcf._lib.tpcf_last_error(None) is not None
    tpcf._lib.tpcf_destroy(None)


def test_sphere_catalog_validation_on_host():
    c = _ctx()
    v = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.6, 0.8]])
    x, y, z = v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
    assert _code(c.set_sphere_catalog, x * 1.001, y, z) == 1  # not unit vectors
    assert "unit vector" in tpcf._lib.tpcf_last_error(c._h).decode()
    assert _code(c.set_sphere_catalog, np.array([1.0, np.nan, 0.0]), y, z) == 1
    assert _code(c.set_sphere_catalog, x, y, z, np.array([1.0, np.inf, 1.0])) == 1
    with pytest.raises(ValueError):
        c.set_sphere_catalog(x, y, z[:2])
    assert tpcf._lib.tpcf_set_sphere_catalog(c._h, -1, None, None, None, None, 0) == 1
    assert tpcf._lib.tpcf_set_sphere_catalog(c._h, 3, None, None, None, None, 0) == 1
    assert tpcf._lib.tpcf_set_sphere_catalog(c._h, 0, None, None, None, None, 5) == 1
    # angular bins beyond pi
    c.set_bins(4, 0.0, 3.5, 2)
    assert _code(c.set_sphere_catalog, x, y, z) == 1
    assert "pi" in tpcf._lib.tpcf_last_error(c._h).decode()


def test_pivot_cell_validation_on_host():
    c = _ctx()
    assert _code(c.set_pivot_cell, float("nan")) == 1
    assert _code(c.set_pivot_cell, float("inf")) == 1
    c.set_pivot_cell(2.5)
    c.set_pivot_cell(-1.0)
    c.set_pivot_cell(0.0)
    assert tpcf._lib.tpcf_set_pivot_cell(None, 1.0) == 1


def test_one_call_forms_marshal_catalogues():
    """Host-side marshalling of the one-call batch forms: offsets, concatenation, unit weights for a
    catalogue given without them, [N, 3] positions split into columns."""
    rng = np.random.default_rng(1)
    a = rng.random((5, 3))
    b = [rng.random(3) for _ in range(3)]
    wb = rng.random(3)
    off, x, y, z, w = tpcf._concat([(a, None), (b[0], b[1], b[2], wb), (b[0], b[1], b[2])])
    np.testing.assert_array_equal(off, [0, 5, 8, 11])
    np.testing.assert_array_equal(x, np.concatenate([a[:, 0], b[0], b[0]]))
    np.testing.assert_array_equal(z, np.concatenate([a[:, 2], b[2], b[2]]))
    np.testing.assert_array_equal(w, np.concatenate([np.ones(5), wb, np.ones(3)]))
    off, x, y, z, w = tpcf._concat([(b[0], b[1], b[2])])
    assert w is None and list(off) == [0, 3]
    with pytest.raises(ValueError):
        tpcf._columns(rng.random((4, 2)))
    with pytest.raises(ValueError):
        tpcf._concat([(b[0],)])


_LOG_CHILD = """
import paper_2604_08855_amd as tpcf
c = tpcf.Context(0)
try:
    c.set_bins(0, 1.0, 2.0, 2)
except tpcf.TpcfError:
    pass
"""


def test_log_levels(tmp_path):
    """TPCF_LOG_LEVEL: 0 (default) prints nothing, 1 reports each failing call with its status and
    message on stderr; TPCF_LOG_FILE sends the lines to a file instead."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def run(**env):
        e = dict(os.environ)
        e.pop("TPCF_LOG_LEVEL", None)
        e.pop("TPCF_LOG_FILE", None)
        e.update(env)
        return subprocess.run([sys.executable, "-c", _LOG_CHILD], cwd=root, env=e, capture_output=True, text=True,
                              timeout=120)

    quiet = run()
    assert quiet.returncode == 0 and "tpcf[" not in quiet.stderr
    loud = run(TPCF_LOG_LEVEL="1")
    assert loud.returncode == 0
    assert "tpcf[error] status 1: nbins" in loud.stderr, loud.stderr
    path = tmp_path / "tpcf.log"
    filed = run(TPCF_LOG_LEVEL="3", TPCF_LOG_FILE=str(path))
    assert "tpcf[" not in filed.stderr
    assert "tpcf[error] status 1: nbins" in path.read_text()
