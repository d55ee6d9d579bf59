"""Batch form: several independent catalogues in one persistent launch (and its HIP graph)."""
import os

import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "mixed": 1e-5}
NB, RMIN, RMAX, L = 8, 3.0, 40.0, 6


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available()
    import paper_2604_08855_amd as mod

    return mod


def make_batch(seed):
    """Uneven mocks: sizes 0, 1, 700, 2500, 4100; different boxes and periodicity."""
    specs = [(0, 100.0, True), (1, 100.0, True), (700, 90.0, False), (2500, 120.0, True), (4100, 150.0, True)]
    cats = []
    for k, (n, box, per) in enumerate(specs):
        if n >= 2500:
            c = catalogs.lognormal(n, box, seed + k, grid=32, periodic=per)
        else:
            c = catalogs.uniform(n, box, seed + k)
            c.periodic = per
        c.w = catalogs.gaussian_weights(n, 100 + seed + k)
        cats.append(c)
    return cats


def concat(cats):
    off = np.concatenate([[0], np.cumsum([c.n for c in cats])]).astype(np.int64)
    cat = lambda f: np.concatenate([getattr(c, f) for c in cats])
    return off, cat("x"), cat("y"), cat("z"), cat("w")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle_per_catalogue(tpcf, prec):
    cats = make_batch(3)
    off, x, y, z, w = concat(cats)
    ctx = tpcf.Context(0)
    ctx.set_bins(NB, RMIN, RMAX, L)
    ctx.set_precision(prec)
    say(f"batch of {len(cats)} catalogues, {off[-1]} points, prec={prec}")
    zb = ctx.compute_batch(off, x, y, z, w, [c.box for c in cats], [c.periodic for c in cats])
    assert zb.shape == (len(cats), L + 1, NB, NB)
    npairs, dd = ctx.pair_sums()
    assert npairs.shape == (len(cats), NB)
    for k, c in enumerate(cats):
        ref = oracle.zeta(c.x, c.y, c.z, c.w, c.box, c.periodic, NB, RMIN, RMAX, L).zeta
        rn, rdd = oracle.pair_sums(c.x, c.y, c.z, c.w, c.box, c.periodic, NB, RMIN, RMAX)
        np.testing.assert_array_equal(npairs[k], rn)
        if rn.any():
            assert np.max(np.abs(dd[k] - rdd)) <= (1e-12 if prec == "fp64" else 2e-6) * np.max(np.abs(rdd))
        if c.n < 2:
            assert not zb[k].any()
            continue
        err = rel_err_per_l(zb[k], ref)
        say(k, c.n, err.max())
        assert err.max() <= TOL[prec], k


def test_graph_replays_match_eager(tpcf):
    """The captured graph is replayed several times on new data, with eager work and
    synchronisations in between; every replay must equal the eager result."""
    import torch

    stream = torch.cuda.Stream()
    ctx = tpcf.Context(0, stream)
    ctx.set_bins(NB, RMIN, RMAX, L)
    ctx.set_precision("mixed")
    other = tpcf.Context(0)
    other.set_bins(NB, RMIN, RMAX, L)
    other.set_precision("fp64")
    for rep in range(4):
        cats = make_batch(10 + rep)  # same shape, new data every time
        off, x, y, z, w = concat(cats)
        boxes, per = [c.box for c in cats], [c.periodic for c in cats]
        os.environ["TPCF_GRAPH"] = "1"
        zg = ctx.compute_batch(off, x, y, z, w, boxes, per)
        # unrelated eager work on another context and torch work in between
        one = cats[3]
        other.set_catalog(one.x, one.y, one.z, one.w, box=one.box, periodic=one.periodic)
        other.compute_zeta()
        torch.ones(1000, device="cuda").sum().item()
        torch.cuda.synchronize()
        os.environ["TPCF_GRAPH"] = "0"
        eager = tpcf.Context(0, stream)
        eager.set_bins(NB, RMIN, RMAX, L)
        eager.set_precision("mixed")
        ze = eager.compute_batch(off, x, y, z, w, boxes, per)
        eager.close()
        os.environ["TPCF_GRAPH"] = "1"
        for k in range(len(cats)):
            if cats[k].n < 2:
                assert not zg[k].any()
                continue
            assert rel_err_per_l(zg[k], ze[k]).max() < 1e-6, (rep, k)
        say(f"replay {rep} ok")


def test_batch_equals_single_runs(tpcf):
    cats = make_batch(21)
    off, x, y, z, w = concat(cats)
    ctx = tpcf.Context(0)
    ctx.set_bins(NB, RMIN, RMAX, L)
    ctx.set_precision("fp64")
    zb = ctx.compute_batch(off, x, y, z, w, [c.box for c in cats], [c.periodic for c in cats])
    for k, c in enumerate(cats):
        s = tpcf.Context(0)
        s.set_bins(NB, RMIN, RMAX, L)
        s.set_precision("fp64")
        s.set_catalog(c.x, c.y, c.z, c.w, box=c.box, periodic=c.periodic)
        zs = s.compute_zeta()
        if c.n < 2:
            assert not zs.any() and not zb[k].any()
        else:
            assert rel_err_per_l(zb[k], zs).max() < 1e-12


def test_batch_at_full_mock_sizes(tpcf):
    """The batch recipe at full size for its first 6 mocks (seeds 0..5, sizes from the C4 size
    stream: log-uniform in [2e5, 2e6]), L = 1000, 20 bins [10, 200), l_max = 10, mixed, in the
    bench's configuration (graph on a stream): each batch slice against a single run of the same
    mock (the single path is checked against the oracle at this size elsewhere), and the batch's
    pair total against the single runs' totals."""
    import torch

    sizes = catalogs.mock_sizes(256, 2e5, 2e6, 1000)[:6]
    cats = [catalogs.lognormal(int(n), 1000.0, i, grid=256) for i, n in enumerate(sizes)]
    say(f"mock sizes {list(map(int, sizes))}")
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat_all = [np.concatenate([getattr(c, a) for c in cats]) for a in ("x", "y", "z")]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = tpcf.Context(0, stream)
        ctx.set_bins(20, 10.0, 200.0, 10)
        ctx.set_precision("mixed")
        dev = [torch.from_numpy(a).cuda() for a in cat_all]
        zb = ctx.compute_batch(off, *dev, None, 1000.0, True).cpu().numpy()
        pairs_b = ctx.stats()["n_pairs"]
    torch.cuda.synchronize()
    total = 0
    for k, c in enumerate(cats):
        s = tpcf.Context(0)
        s.set_bins(20, 10.0, 200.0, 10)
        s.set_precision("mixed")
        s.set_catalog(c.x, c.y, c.z, None, box=1000.0, periodic=True)
        zs = s.compute_zeta()
        total += s.stats()["n_pairs"]
        err = rel_err_per_l(zb[k], zs).max()
        say(f"mock {k}: n={c.n} batch vs single {err:.2e}")
        assert err < 1e-6
    assert pairs_b == total


def test_one_call_forms(tpcf):
    """tpcf.zeta with [N, 3] positions, tpcf.zeta_batch over catalogues given in the three accepted
    forms, and tpcf.zeta_sphere_batch over two maps, each against the oracle."""
    a = catalogs.uniform(2000, 150.0, 301)
    b = catalogs.uniform(1500, 150.0, 302)
    c = catalogs.uniform(2500, 150.0, 303)
    wb = catalogs.gaussian_weights(b.n, 304, 1.0, 0.3)
    say("one-call forms")
    pos = np.stack([a.x, a.y, a.z], 1)
    z1 = tpcf.zeta(pos, box=150.0, periodic=True, rmin=4.0, rmax=30.0, nbins=6, lmax=3)
    r1 = oracle.zeta(a.x, a.y, a.z, None, 150.0, True, 6, 4.0, 30.0, 3)
    assert rel_err_per_l(z1, r1.zeta).max() <= 1e-10
    zb = tpcf.zeta_batch([(pos, None), (b.x, b.y, b.z, wb), (c.x, c.y, c.z)], box=150.0, periodic=[True, False, True],
                         rmin=4.0, rmax=30.0, nbins=6, lmax=3)
    assert zb.shape == (3, 4, 6, 6)
    refs = [r1.zeta, oracle.zeta(b.x, b.y, b.z, wb, 150.0, False, 6, 4.0, 30.0, 3).zeta,
            oracle.zeta(c.x, c.y, c.z, None, 150.0, True, 6, 4.0, 30.0, 3).zeta]
    for k in range(3):
        assert rel_err_per_l(zb[k], refs[k]).max() <= 1e-5
    maps = [catalogs.sphere_map(16, 7 + k, grid=32) for k in range(2)]
    zs = tpcf.zeta_sphere_batch([(m.x, m.y, m.z, m.w) for m in maps], theta_min=0.05, theta_max=0.4, nbins=5,
                                mmax=4)
    for k, m in enumerate(maps):
        ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 5, 0.05, 0.4, 4).zeta
        assert rel_err_per_l(zs[k], ref).max() <= 1e-5

