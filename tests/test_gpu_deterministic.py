"""Deterministic mode (tpcf_set_deterministic): fixed contraction tiles and a fixed-order reduction
make the result bit-for-bit reproducible, independent of how many waves run and which wave takes
which tile, and it stays within the usual bars of the FP64 oracle (FP64 1e-10, mixed 1e-5 per l).
Pair counts are exact either way.
"""
import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say
from tests.test_gpu_batch import concat, make_batch

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available()
    import paper_2604_08855_amd as mod

    return mod


def det_ctx(tpcf, prec, nb, rmin, rmax, lmax, waves=0, det=True):
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    ctx.set_deterministic(det)
    if waves:
        ctx.set_tuning(0.0, waves)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_config_bit_identical(tpcf, prec):
    """10,000 uniform points in a periodic box of 250, 10 bins [5, 50), l_max = 4, weights
    1 + 0.1 N(0,1): three deterministic runs, with 12, 3 and 1 waves per compute unit, give the same
    bits for zeta and the 2PCF weight sums; they match the oracle, and the atomic (default) mode
    agrees with them within the bar."""
    cat = catalogs.uniform(10000, 250.0, 0)
    w = catalogs.gaussian_weights(cat.n, 7)
    say(f"deterministic small config prec={prec}")
    runs = []
    for waves in (12, 3, 1):
        ctx = det_ctx(tpcf, prec, 10, 5.0, 50.0, 4, waves)
        ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
        z = ctx.compute_zeta()
        runs.append((z, ctx.pair_sums()))
    for z, (n, dd) in runs[1:]:
        assert np.array_equal(z, runs[0][0])
        assert np.array_equal(n, runs[0][1][0]) and np.array_equal(dd, runs[0][1][1])
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 10, 5.0, 50.0, 4)
    err = rel_err_per_l(runs[0][0], ref.zeta)
    say("rel err per l", err)
    assert err.max() <= TOL[prec]
    ctx = det_ctx(tpcf, prec, 10, 5.0, 50.0, 4, det=False)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
    assert rel_err_per_l(ctx.compute_zeta(), runs[0][0]).max() <= TOL[prec]
    assert ctx.stats()["n_pairs"] == ref.npairs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_bit_identical(tpcf, prec):
    """A batch of five uneven catalogues (sizes 0 to 4100, periodic and not): two deterministic
    runs with different wave counts agree bit for bit, and every catalogue matches the oracle."""
    cats = make_batch(11)
    off, x, y, z, w = concat(cats)
    out = []
    for waves in (12, 2):
        ctx = det_ctx(tpcf, prec, 8, 3.0, 30.0, 6, waves)
        out.append(ctx.compute_batch(off, x, y, z, w, [c.box for c in cats], [c.periodic for c in cats]))
    assert np.array_equal(out[0], out[1])
    for k, c in enumerate(cats):
        ref = oracle.zeta(c.x, c.y, c.z, c.w, c.box, c.periodic, 8, 3.0, 30.0, 6).zeta
        if np.abs(ref).max() == 0.0:
            assert not out[0][k].any()
            continue
        assert rel_err_per_l(out[0][k], ref).max() <= TOL[prec]


def test_range_and_degenerate_bit_identical(tpcf):
    """A primary range and the degenerate term are reproducible too (log-normal catalogue)."""
    cat = catalogs.lognormal(6000, 200.0, 21, grid=32)
    w = catalogs.gaussian_weights(cat.n, 22)
    zs, ds = [], []
    for waves in (12, 5):
        ctx = det_ctx(tpcf, "mixed", 10, 4.0, 50.0, 6, waves)
        ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
        zs.append(ctx.compute_zeta_range(1000, 3500))
        ds.append(ctx.degenerate())
    assert np.array_equal(zs[0], zs[1]) and np.array_equal(ds[0], ds[1])
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 10, 4.0, 50.0, 6, 1000, 3500).zeta
    assert rel_err_per_l(zs[0], ref).max() <= TOL["mixed"]
    dref = oracle.degenerate(cat.x, cat.y, cat.z, w, cat.box, True, 10, 4.0, 50.0, 6)
    assert np.abs(ds[0] - dref).max() <= 1e-10 * np.abs(dref).max()


@pytest.mark.parametrize("ppc", [400.0, 40000.0])
def test_large_cells_sorted(tpcf, ppc):
    """Cells far above the usual occupancy (about 100 points with 400 per cell, several thousand
    with 40000: one cell across y and z, split four ways along x) go through the in-LDS bitonic
    sort or the workgroup rank count; their in-cell order is the input order, so deterministic runs
    still agree bit for bit, and counts and zeta match the oracle."""
    cat = catalogs.uniform(20000, 100.0, 5)
    w = catalogs.gaussian_weights(cat.n, 6)
    zs = []
    for waves in (12, 4):
        ctx = det_ctx(tpcf, "fp64", 6, 2.0, 20.0, 3, waves)
        ctx.set_tuning(ppc, waves)
        ctx.set_debug(True)
        ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
        zs.append(ctx.compute_zeta())
    say("cells per axis", ctx.stats()["cells_per_axis"])
    assert np.array_equal(zs[0], zs[1])
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 6, 2.0, 20.0, 3, want_counts=True)
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    assert rel_err_per_l(zs[0], ref.zeta).max() <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sphere_bit_identical(tpcf, prec):
    """A HEALPix nside-32 map (12,288 pixels, log-normal values), 8 angular bins in [0.02, 0.3)
    rad, m_max = 6: deterministic runs with 12 and 3 waves per CU give the same bits, and match
    the sphere oracle."""
    m = catalogs.sphere_map(32, 5, grid=32)
    zs = []
    for waves in (12, 3):
        ctx = det_ctx(tpcf, prec, 8, 0.02, 0.3, 6, waves)
        ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
        zs.append(ctx.compute_zeta())
    assert np.array_equal(zs[0], zs[1])
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 8, 0.02, 0.3, 6).zeta
    assert rel_err_per_l(zs[0], ref).max() <= TOL[prec]


def test_shared_pivots_bit_identical(tpcf):
    """Shared pivots (cells of 3, 6,000 log-normal points, signed weights): the deterministic
    pivot sweep gives the same bits with 12 and 4 waves per CU and matches the pivot oracle."""
    cat = catalogs.lognormal(6000, 150.0, 4, grid=64)
    w = catalogs.gaussian_weights(cat.n, 9, 0.4, 1.0)
    zs = []
    for waves in (12, 4):
        ctx = det_ctx(tpcf, "mixed", 10, 3.0, 30.0, 6, waves)
        ctx.set_pivot_cell(3.0)
        ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
        zs.append(ctx.compute_zeta())
    assert np.array_equal(zs[0], zs[1])
    ref = oracle.zeta_pivots(cat.x, cat.y, cat.z, w, cat.box, True, 10, 3.0, 30.0, 6, 3.0).zeta
    assert rel_err_per_l(zs[0], ref).max() <= TOL["mixed"]
