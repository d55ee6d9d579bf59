"""GPU parity of the degenerate (j = k) term, tpcf_degenerate, against oracle_degenerate and
oracle_degenerate_sphere on identical seeded inputs.

The device computes it as an FP64 sweep, so the bar is the FP64 one: max|D - oracle| per l
<= 1e-10 * max|oracle_l|. The call must leave the last compute call's outputs as they were.
"""
import math

import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_08855_amd as mod

    return mod


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
def test_degenerate_3d(tpcf, prec, periodic):
    """3,001 points, signed weights, 20 bins [3, 45), l_max = 10 (either compute precision: the
    term itself is always FP64); the compute call's zeta and pair sums are unchanged by it."""
    cat = catalogs.uniform(3001, 160.0, 7)
    w = catalogs.gaussian_weights(cat.n, 8, 0.3, 1.0)
    say(f"degenerate 3d periodic={periodic} prec={prec}")
    ctx = tpcf.Context(0)
    ctx.set_bins(20, 3.0, 45.0, 10)
    ctx.set_precision(prec)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=periodic)
    z = ctx.compute_zeta()
    np0, dd0 = ctx.pair_sums()
    st0 = ctx.stats()
    D = ctx.degenerate()
    ref = oracle.degenerate(cat.x, cat.y, cat.z, w, cat.box, periodic, 20, 3.0, 45.0, 10)
    assert D.shape == (1, 11, 20)
    for l in range(11):
        assert _rel(D[0, l], ref[l]) <= TOL, l
    np1, dd1 = ctx.pair_sums()
    np.testing.assert_array_equal(np1, np0)
    np.testing.assert_array_equal(dd1, dd0)
    assert ctx.stats()["n_pairs"] == st0["n_pairs"]
    z2 = ctx.compute_zeta()  # the next compute call runs at the context's own l_max and precision
    assert np.abs(z2 - z).max() <= 1e-5 * np.abs(z).max()


def test_degenerate_worked_triangle(tpcf):
    """Three points O, O + 10 x, O + 10 y: zeta_l(2, 2) - D_l(2) = 0 and zeta_l(1, 1) - D_l(1) =
    2 c_l P_l(0), the one triangle of distinct points (both orders) on bin 1."""
    from scipy.special import eval_legendre

    x = np.array([125.0, 135.0, 125.0])
    y = np.array([125.0, 125.0, 135.0])
    z = np.full(3, 125.0)
    ctx = tpcf.Context(0)
    ctx.set_bins(10, 5.0, 50.0, 4)
    ctx.set_precision("fp64")
    ctx.set_catalog(x, y, z, None, box=250.0, periodic=True)
    zt = ctx.compute_zeta()
    D = ctx.degenerate()[0]
    for l in range(5):
        c = (2 * l + 1) / (4 * math.pi)
        assert abs(zt[l, 2, 2] - D[l, 2]) < 1e-14
        assert abs(zt[l, 1, 1] - D[l, 1] - 2 * c * eval_legendre(l, 0.0)) < 1e-13
        assert abs(D[l, 1] - 4 * c) < 1e-14 and abs(D[l, 2] - 2 * c) < 1e-14


def test_degenerate_sphere(tpcf):
    """HEALPix nside 32 map with signed values, 10 bins [0.02, 0.3) rad, m_max = 8: D_m(b) the
    same for every m and equal to the oracle's."""
    m = catalogs.sphere_map(32, 5, grid=64)
    say("degenerate sphere nside=32")
    ctx = tpcf.Context(0)
    ctx.set_bins(10, 0.02, 0.3, 8)
    ctx.set_precision("mixed")
    ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
    ctx.compute_zeta()
    D = ctx.degenerate()[0]
    ref = oracle.degenerate_sphere(m.x, m.y, m.z, m.w, 10, 0.02, 0.3, 8)
    assert _rel(D, ref) <= TOL
    for k in range(9):
        np.testing.assert_array_equal(D[k], D[0])


def test_degenerate_batch_and_pivots(tpcf):
    """A batch of three catalogues (one of a single point) per catalogue against the oracle; with
    shared pivots set the term is still the exact one."""
    cats = [catalogs.uniform(n, 200.0, 60 + k) for k, n in enumerate((2500, 1, 4000))]
    ws = [catalogs.gaussian_weights(c.n, 70 + k, 0.5, 1.0) for k, c in enumerate(cats)]
    off = np.cumsum([0] + [c.n for c in cats]).astype(np.int64)
    x, y, z = (np.concatenate([getattr(c, a) for c in cats]) for a in "xyz")
    w = np.concatenate(ws)
    say("degenerate batch")
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 5.0, 40.0, 4)
    ctx.set_precision("mixed")
    ctx.compute_batch(off, x, y, z, w, [200.0] * 3, [True] * 3)
    D = ctx.degenerate()
    assert D.shape == (3, 5, 8)
    for k, c in enumerate(cats):
        ref = oracle.degenerate(c.x, c.y, c.z, ws[k], c.box, True, 8, 5.0, 40.0, 4)
        if np.abs(ref).max() == 0.0:
            assert np.abs(D[k]).max() == 0.0
        else:
            assert _rel(D[k], ref) <= TOL
    say("degenerate with pivots set")
    c, wc = cats[2], ws[2]
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 5.0, 40.0, 4)
    ctx.set_pivot_cell(12.0)
    ctx.set_catalog(c.x, c.y, c.z, wc, box=c.box, periodic=True)
    ctx.compute_zeta()
    ref = oracle.degenerate(c.x, c.y, c.z, wc, c.box, True, 8, 5.0, 40.0, 4)
    assert _rel(ctx.degenerate()[0], ref) <= TOL


def test_degenerate_empty_catalogue(tpcf):
    ctx = tpcf.Context(0)
    ctx.set_bins(5, 1.0, 10.0, 2)
    ctx.set_catalog(np.zeros(0), np.zeros(0), np.zeros(0), None, box=50.0, periodic=True)
    assert np.abs(ctx.compute_zeta()).max() == 0.0
    D = ctx.degenerate()
    assert D.shape == (1, 3, 5) and np.abs(D).max() == 0.0

