"""GPU parity with phase-aligned stencil sweeps forced on (tpcf_set_phase_aligned(ctx, 1)).

The rotation changes only the order in which a wave visits its stencil rows: per-primary per-bin
pair counts stay bit-exact against the oracle, zeta keeps the usual bars (FP64 1e-10, mixed 1e-5
of max|oracle_l| per l) and agrees with the unrotated sweep to the same bars. Fine grids (few
points per cell) give stencils of several 64-row chunks, so the chunk search and the wrap-around
are both exercised.
"""
import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_08855_amd as mod

    return mod


def run(tpcf, setup, phase, prec, nb, rmin, rmax, lmax, ppc, prange=None):
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    ctx.set_tuning(ppc)
    ctx.set_phase_aligned(phase)
    ctx.set_debug(True)
    setup(ctx)
    z = ctx.compute_zeta() if prange is None else ctx.compute_zeta_range(*prange)
    return ctx, z


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
def test_phase_aligned_3d(tpcf, prec, periodic):
    """20,000 uniform points, box 250, 12 bins [4, 50), l_max = 6, signed weights; 2 points per
    cell: 21 cells per axis, stencils of 13 x 13 rows (3 chunks)."""
    cat = catalogs.uniform(20000, 250.0, 31)
    cat.periodic = periodic
    w = catalogs.gaussian_weights(cat.n, 32, 0.3, 1.0)
    say(f"phase 3d periodic={periodic} prec={prec}")

    def setup(ctx):
        ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=periodic)

    on, zon = run(tpcf, setup, 1, prec, 12, 4.0, 50.0, 6, 2.0)
    off, zoff = run(tpcf, setup, 0, prec, 12, 4.0, 50.0, 6, 2.0)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, periodic, 12, 4.0, 50.0, 6, want_counts=True)
    err = rel_err_per_l(zon, ref.zeta)
    say("rel err per l (aligned)", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(on.pair_counts(), ref.counts)
    assert on.stats()["n_pairs"] == off.stats()["n_pairs"] == ref.npairs
    assert on.stats()["n_candidates"] == off.stats()["n_candidates"]
    assert rel_err_per_l(zon, zoff).max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_phase_aligned_sphere(tpcf, prec):
    """HEALPix nside 32 with log-normal map values, 10 bins [0.02, 0.3) rad, m_max = 8; 1 point
    per cell: 19 x 19 stencil rows (6 chunks, the last one partial)."""
    m = catalogs.sphere_map(32, 5, grid=64)
    say(f"phase sphere nside=32 prec={prec}")

    def setup(ctx):
        ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)

    on, zon = run(tpcf, setup, 1, prec, 10, 0.02, 0.3, 8, 1.0)
    off, zoff = run(tpcf, setup, 0, prec, 10, 0.02, 0.3, 8, 1.0)
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 10, 0.02, 0.3, 8, want_counts=True)
    err = rel_err_per_l(zon, ref.zeta)
    say("rel err per m (aligned)", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(on.pair_counts(), ref.counts)
    assert on.stats()["n_pairs"] == off.stats()["n_pairs"] == ref.npairs
    assert rel_err_per_l(zon, zoff).max() <= TOL[prec]


def test_phase_aligned_range_and_batch(tpcf):
    """A primary range (tickets restart at 0, fewer tasks than waves) and a batch of three
    catalogues with alignment on: each against the oracle."""
    cat = catalogs.uniform(6000, 200.0, 41)
    say("phase range")

    def setup(ctx):
        ctx.set_catalog(cat.x, cat.y, cat.z, None, box=cat.box, periodic=True)

    ctx, z = run(tpcf, setup, 1, "fp64", 8, 5.0, 40.0, 4, 2.0, prange=(1000, 1777))
    ref = oracle.zeta(cat.x, cat.y, cat.z, None, cat.box, True, 8, 5.0, 40.0, 4, 1000, 1777)
    assert rel_err_per_l(z, ref.zeta).max() <= TOL["fp64"]

    say("phase batch")
    cats = [catalogs.uniform(n, 200.0, 50 + k) for k, n in enumerate((3000, 1, 4500))]
    off = np.cumsum([0] + [c.n for c in cats]).astype(np.int64)
    x, y, zz = (np.concatenate([getattr(c, a) for c in cats]) for a in "xyz")
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 5.0, 40.0, 4)
    ctx.set_precision("mixed")
    ctx.set_tuning(2.0)
    ctx.set_phase_aligned(1)
    zb = ctx.compute_batch(off, x, y, zz, None, [200.0] * 3, [True] * 3)
    for k, c in enumerate(cats):
        ref = oracle.zeta(c.x, c.y, c.z, None, c.box, True, 8, 5.0, 40.0, 4)
        if np.abs(ref.zeta).max() == 0.0:
            assert np.abs(zb[k]).max() == 0.0
        else:
            assert rel_err_per_l(zb[k], ref.zeta).max() <= TOL["mixed"]


def test_phase_aligned_beyond_64_row_chunks(tpcf):
    """A stencil of more than 64 row chunks (0.005 points per cell: 158 cells per axis, 67 x 67 =
    4,489 rows) keeps its natural row order, as documented; results as usual."""
    cat = catalogs.uniform(20000, 250.0, 45)
    say("phase: stencil beyond 4096 rows")

    def setup(ctx):
        ctx.set_catalog(cat.x, cat.y, cat.z, None, box=cat.box, periodic=True)

    on, zon = run(tpcf, setup, 1, "fp64", 6, 4.0, 50.0, 3, 0.005)
    ref = oracle.zeta(cat.x, cat.y, cat.z, None, cat.box, True, 6, 4.0, 50.0, 3, want_counts=True)
    assert rel_err_per_l(zon, ref.zeta).max() <= TOL["fp64"]
    np.testing.assert_array_equal(on.pair_counts(), ref.counts)

