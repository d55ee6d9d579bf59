"""GPU parity of the shared-pivot approximation (tpcf_set_pivot_cell) against the FP64 oracle's
definition of it (oracle_zeta_pivots), at the same bars as the exact estimator: 1e-10 (FP64) and
1e-5 (mixed) of max|zeta_l| per l; pivot and pair counts exact."""
import numpy as np
import pytest

import catalogs
import oracle
from tests import brute
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_08855_amd as mod

    return mod


def run(tpcf, cat, w, nb, rmin, rmax, lmax, prec, side, periodic=None):
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    ctx.set_pivot_cell(side)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=cat.periodic if periodic is None else periodic)
    return ctx, ctx.compute_zeta()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
def test_pivots_match_oracle(tpcf, prec, periodic):
    """6,000 log-normal points, pivot cells of 3 (several points per cell in clusters), signed
    weights, 10 bins in [3, 30), l_max = 6."""
    cat = catalogs.lognormal(6000, 150.0, 4, grid=64)
    cat.periodic = periodic
    w = catalogs.gaussian_weights(cat.n, 9, 0.4, 1.0)
    say(f"pivots periodic={periodic} prec={prec}")
    ctx, z = run(tpcf, cat, w, 10, 3.0, 30.0, 6, prec, 3.0)
    ref = oracle.zeta_pivots(cat.x, cat.y, cat.z, w, 150.0, periodic, 10, 3.0, 30.0, 6, 3.0)
    st = ctx.stats()
    say("groups", ref.ngroups, "pairs", ref.npairs, "rel err", rel_err_per_l(z, ref.zeta).max())
    assert st["n_primaries"] == ref.ngroups < cat.n
    assert st["n_pairs"] == ref.npairs
    assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]
    npairs, _ = ctx.pair_sums()
    assert npairs.sum() == ref.npairs


def test_one_point_per_cell_is_exact(tpcf):
    """Pivot cells so small that each holds one point: the shared-pivot result is the exact one."""
    rng = np.random.default_rng(2)
    cells = rng.choice(40 ** 3, 3000, replace=False)
    ijk = np.stack(np.unravel_index(cells, (40, 40, 40)), 1)
    P = (ijk + 0.1 + 0.8 * rng.random((3000, 3))) * 2.5
    cat = catalogs.Catalog(P[:, 0], P[:, 1], P[:, 2], np.ones(3000), 100.0, True)
    w = catalogs.gaussian_weights(cat.n, 3, 1.0, 0.2)
    ctx, z = run(tpcf, cat, w, 8, 2.0, 20.0, 5, "fp64", 2.5 * (1 + 1e-12))
    ex = tpcf.Context(0)
    ex.set_bins(8, 2.0, 20.0, 5)
    ex.set_catalog(cat.x, cat.y, cat.z, w, box=100.0, periodic=True)
    ze = ex.compute_zeta()
    assert ctx.stats()["n_primaries"] == cat.n
    assert rel_err_per_l(z, ze).max() < 1e-12


def test_mean_separation_default_and_errors(tpcf):
    """side < 0 uses the mean separation L / n^(1/3); ranges and more than 2^21 pivot cells per
    axis are refused."""
    cat = catalogs.lognormal(4000, 120.0, 6, grid=64)
    ctx, z = run(tpcf, cat, None, 6, 4.0, 24.0, 3, "fp64", -1.0)
    h = 120.0 / np.cbrt(4000.0)
    ref = oracle.zeta_pivots(cat.x, cat.y, cat.z, None, 120.0, True, 6, 4.0, 24.0, 3, h)
    assert ctx.stats()["n_primaries"] == ref.ngroups
    assert rel_err_per_l(z, ref.zeta).max() <= TOL["fp64"]
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.compute_zeta_range(0, 10)
    assert e.value.code == 5
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.set_pivot_cell(float("nan"))
    assert e.value.code == 1
    ctx.set_pivot_cell(1e-5)  # 1.2e7 cells per axis, above 2^21
    ctx.set_catalog(cat.x, cat.y, cat.z, None, box=120.0, periodic=True)
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.compute_zeta()
    assert e.value.code == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sphere_pivots_match_oracle(tpcf, prec):
    """Shared pivots on a HEALPix nside-32 map (12,288 pixels, mean separation 0.032): cells of
    0.06, 10 bins in [0.02, 0.3) rad, m_max = 8; and the sphere's mean-separation default."""
    m = catalogs.sphere_map(32, 5, grid=64)
    for side, h in ((0.06, 0.06), (-1.0, np.sqrt(4 * np.pi / m.n))):
        ctx = tpcf.Context(0)
        ctx.set_bins(10, 0.02, 0.3, 8)
        ctx.set_precision(prec)
        ctx.set_pivot_cell(side)
        ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
        z = ctx.compute_zeta()
        ref = oracle.zeta_sphere_pivots(m.x, m.y, m.z, m.w, 10, 0.02, 0.3, 8, h)
        st = ctx.stats()
        say(f"sphere pivots side={side} prec={prec}: {st['n_primaries']} pivots, rel err",
            rel_err_per_l(z, ref.zeta).max())
        assert st["n_primaries"] == ref.ngroups and st["n_pairs"] == ref.npairs
        assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]
    ctx.set_pivot_cell(0.3)  # cells comparable with the radius: refused
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.compute_zeta()
    assert e.value.code == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_pivots_match_oracle(tpcf, prec):
    """Shared pivots over a batch: four catalogues (clustered and periodic, one point, none,
    uniform and non-periodic with another box), pivot cells of 3 and the per-catalogue
    mean-separation default. Every catalogue's pivots stay its own (cells never merge across
    catalogues, even where the boxes overlap); each zeta against oracle_zeta_pivots."""
    cats = [catalogs.lognormal(4000, 120.0, 21, grid=64), catalogs.uniform(1, 120.0, 22),
            catalogs.uniform(0, 120.0, 23), catalogs.uniform(2500, 150.0, 24)]
    per = [True, True, True, False]
    ws = [catalogs.gaussian_weights(c.n, 30 + k, 0.4, 1.0) for k, c in enumerate(cats)]
    off = np.cumsum([0] + [c.n for c in cats]).astype(np.int64)
    x, y, z = (np.concatenate([getattr(c, a) for c in cats]) for a in "xyz")
    w = np.concatenate(ws)
    for side in (3.0, -1.0):
        say(f"batch pivots side={side} prec={prec}")
        ctx = tpcf.Context(0)
        ctx.set_bins(8, 3.0, 24.0, 4)
        ctx.set_precision(prec)
        ctx.set_pivot_cell(side)
        zb = ctx.compute_batch(off, x, y, z, w, [c.box for c in cats], per)
        groups = pairs = 0
        for k, c in enumerate(cats):
            h = side if side > 0 else (c.box / np.cbrt(c.n) if c.n else c.box)
            ref = oracle.zeta_pivots(c.x, c.y, c.z, ws[k], c.box, per[k], 8, 3.0, 24.0, 4, h)
            groups += ref.ngroups
            pairs += ref.npairs
            if np.abs(ref.zeta).max() == 0.0:
                assert np.abs(zb[k]).max() == 0.0
            else:
                assert rel_err_per_l(zb[k], ref.zeta).max() <= TOL[prec], k
        st = ctx.stats()
        assert st["n_primaries"] == groups and st["n_pairs"] == pairs
        npairs, _ = ctx.pair_sums()
        assert npairs.sum() == pairs


def test_sphere_batch_pivots_match_oracle(tpcf):
    """Shared pivots over a batch of two HEALPix nside-16 maps (cells of 0.08), per map against
    oracle_zeta_sphere_pivots."""
    maps = [catalogs.sphere_map(16, 40 + k, grid=32) for k in range(2)]
    off = np.cumsum([0] + [m.n for m in maps]).astype(np.int64)
    x, y, z, w = (np.concatenate([getattr(m, a) for m in maps]) for a in ("x", "y", "z", "w"))
    ctx = tpcf.Context(0)
    ctx.set_bins(6, 0.05, 0.4, 6)
    ctx.set_precision("mixed")
    ctx.set_pivot_cell(0.08)
    zb = ctx.compute_sphere_batch(off, x, y, z, w)
    for k, m in enumerate(maps):
        ref = oracle.zeta_sphere_pivots(m.x, m.y, m.z, m.w, 6, 0.05, 0.4, 6, 0.08)
        assert rel_err_per_l(zb[k], ref.zeta).max() <= TOL["mixed"]


def test_full_size_pivots(tpcf):
    """The benchmark catalogue (10^6 log-normal points, L = 1000, 20 bins [10, 200), l_max = 10)
    with pivot cells of the mean separation (10): pivot count against the numpy grouping, and
    zeta within 2% of the exact estimator per l (mixed)."""
    cat = catalogs.lognormal(10**6, 1000.0, 0, grid=256)
    w = catalogs.gaussian_weights(cat.n, 10**6, 1.0, 0.1)
    ctx, z = run(tpcf, cat, w, 20, 10.0, 200.0, 10, "mixed", 10.0)
    st = ctx.stats()
    X, W, _, _ = brute.pivot_groups(cat.x, cat.y, cat.z, w, 1000.0, True, 200.0, 10.0)
    say(f"pivots: {st['n_primaries']} (numpy {len(X)}), sweep {st['ms_sweep']:.1f} ms")
    assert st["n_primaries"] == len(X)
    ex = tpcf.Context(0)
    ex.set_bins(20, 10.0, 200.0, 10)
    ex.set_precision("mixed")
    ex.set_catalog(cat.x, cat.y, cat.z, w, box=1000.0, periodic=True)
    ze = ex.compute_zeta()
    err = rel_err_per_l(z, ze)
    say("rel err vs exact per l", err, "exact sweep", ex.stats()["ms_sweep"])
    assert err.max() < 0.02
