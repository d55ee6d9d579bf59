"""GPU parity over seeded random configurations: catalogue size (0 to 2,500, including 1), box,
bins (1 to 32), l_max (0 to 10), periodic or not, signed or unit weights, precision, grid density
and phase alignment in 3D; map resolution, angular range up to 1 rad and m_max on the sphere.
Every case: per-primary pair counts bit-exact and zeta at the usual bars (FP64 1e-10, mixed 1e-5
of max|oracle_l|) against the oracle. The seeds are fixed, so the cases are the same every run."""
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


def _check(ctx, z, ref, prec, what):
    if np.abs(ref.zeta).max() == 0.0:
        assert np.abs(z).max() == 0.0, what
    else:
        err = rel_err_per_l(z, ref.zeta).max()
        assert err <= TOL[prec], (what, err)
    if ref.counts is not None and len(ref.counts):
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts, err_msg=what)
    assert ctx.stats()["n_pairs"] == ref.npairs, what


@pytest.mark.parametrize("seed", range(40))
def test_random_3d(tpcf, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(0, 3)) if rng.random() < 0.15 else int(rng.integers(3, 2501))
    box = float(rng.uniform(50.0, 300.0))
    periodic = bool(rng.integers(0, 2))
    rmax = float(rng.uniform(0.03, 0.38) * box)
    rmin = float(rng.uniform(0.0, 0.5) * rmax) if rng.integers(0, 3) else 0.0
    nb = int(rng.integers(1, 33))
    lmax = int(rng.integers(0, 11))
    prec = str(rng.choice(["fp64", "mixed"]))
    ppc = float(rng.choice([0.5, 2.0, 8.0, 32.0]))
    phase = int(rng.integers(-1, 2))
    pos = rng.random((n, 3)) * box
    pos = np.minimum(pos, np.nextafter(box, 0.0))
    w = rng.normal(0.2, 1.0, n) if rng.integers(0, 2) else None
    what = (f"seed={seed} n={n} box={box:.1f} periodic={periodic} r=[{rmin:.2f},{rmax:.2f}) nb={nb} "
            f"lmax={lmax} {prec} ppc={ppc} phase={phase} weights={w is not None}")
    say(what)
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    ctx.set_tuning(ppc)
    ctx.set_phase_aligned(phase)
    ctx.set_debug(True)
    ctx.set_catalog(pos[:, 0], pos[:, 1], pos[:, 2], w, box=box, periodic=periodic)
    z = ctx.compute_zeta()
    ref = oracle.zeta(pos[:, 0], pos[:, 1], pos[:, 2], w, box, periodic, nb, rmin, rmax, lmax, want_counts=True)
    _check(ctx, z, ref, prec, what)


@pytest.mark.parametrize("seed", range(16))
def test_random_sphere(tpcf, seed):
    rng = np.random.default_rng(2000 + seed)
    nside = int(rng.choice([2, 4, 8, 16]))
    m = catalogs.sphere_map(nside, 100 + seed, grid=32)
    tmax = float(rng.uniform(0.05, 1.0))
    tmin = float(rng.uniform(0.0, 0.5) * tmax) if rng.integers(0, 3) else 0.0
    nb = int(rng.integers(1, 33))
    mmax = int(rng.integers(0, 11))
    prec = str(rng.choice(["fp64", "mixed"]))
    ppc = float(rng.choice([1.0, 4.0, 16.0]))
    what = f"seed={seed} nside={nside} theta=[{tmin:.3f},{tmax:.3f}) nb={nb} mmax={mmax} {prec} ppc={ppc}"
    say(what)
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, tmin, tmax, mmax)
    ctx.set_precision(prec)
    ctx.set_tuning(ppc)
    ctx.set_debug(True)
    ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
    z = ctx.compute_zeta()
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, nb, tmin, tmax, mmax, want_counts=True)
    _check(ctx, z, ref, prec, what)


@pytest.mark.parametrize("seed", range(12))
def test_random_batch(tpcf, seed):
    """1 to 5 catalogues with their own boxes, periodicity, sizes (0 included) and weights; exact
    or with shared pivots (a random cell side, or each catalogue's mean separation); zeta and the
    degenerate term of every catalogue against the oracle."""
    rng = np.random.default_rng(3000 + seed)
    ncat = int(rng.integers(1, 6))
    rmax = float(rng.uniform(5.0, 30.0))
    rmin = float(rng.uniform(0.0, 0.5) * rmax)
    nb = int(rng.integers(1, 21))
    lmax = int(rng.integers(0, 9))
    prec = str(rng.choice(["fp64", "mixed"]))
    side = float(rng.choice([0.0, 0.0, -1.0, rng.uniform(1.0, 6.0)]))
    cats = []
    for k in range(ncat):
        n = 0 if rng.random() < 0.1 else int(rng.integers(1, 1500))
        box = float(rng.uniform(2.2 * rmax, 8.0 * rmax))
        per = bool(rng.integers(0, 2))
        pos = np.minimum(rng.random((n, 3)) * box, np.nextafter(box, 0.0))
        w = rng.normal(0.3, 1.0, n)
        cats.append((pos, w, box, per))
    what = f"seed={seed} ncat={ncat} r=[{rmin:.2f},{rmax:.2f}) nb={nb} lmax={lmax} {prec} pivot side={side:.2f}"
    say(what)
    off = np.cumsum([0] + [len(c[0]) for c in cats]).astype(np.int64)
    allpos = np.concatenate([c[0] for c in cats]) if off[-1] else np.zeros((0, 3))
    w = np.concatenate([c[1] for c in cats])
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    ctx.set_pivot_cell(side)
    zb = ctx.compute_batch(off, allpos[:, 0].copy(), allpos[:, 1].copy(), allpos[:, 2].copy(), w,
                           [c[2] for c in cats], [c[3] for c in cats])
    D = ctx.degenerate()
    for k, (pos, wk, box, per) in enumerate(cats):
        x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
        if side != 0.0:
            h = side if side > 0 else (box / np.cbrt(len(pos)) if len(pos) else box)
            ref = oracle.zeta_pivots(x, y, z, wk, box, per, nb, rmin, rmax, lmax, h).zeta
        else:
            ref = oracle.zeta(x, y, z, wk, box, per, nb, rmin, rmax, lmax).zeta
        if np.abs(ref).max() == 0.0:
            assert np.abs(zb[k]).max() == 0.0, (what, k)
        else:
            assert rel_err_per_l(zb[k], ref).max() <= TOL[prec], (what, k)
        Dref = oracle.degenerate(x, y, z, wk, box, per, nb, rmin, rmax, lmax)
        assert np.abs(D[k] - Dref).max() <= 1e-10 * max(np.abs(Dref).max(), 1e-300), (what, k)
