"""GPU parity on the unit sphere: projected fields with 2D multipoles of the position angle.

The HIP path (tpcf_set_sphere_catalog + the compute calls) against the FP64 oracle
(oracle_zeta_sphere) on identical seeded inputs. Bars as for 3D: FP64 path max|zeta_m - oracle_m|
<= 1e-10 * max|oracle_m| per m, mixed path <= 1e-5 * max|oracle_m|; per-primary per-bin pair
counts bit-exact.
"""
import ctypes
import time

import numpy as np
import pytest

import catalogs
import oracle
from tests import brute
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
ARCMIN = np.pi / (180.0 * 60.0)


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_08855_amd as mod

    return mod


def run_sphere(tpcf, m, nb, tmin, tmax, mmax, prec, debug=False, prange=None, tuning=None):
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, tmin, tmax, mmax)
    ctx.set_precision(prec)
    if tuning:
        ctx.set_tuning(*tuning)
    ctx.set_debug(debug)
    ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
    z = ctx.compute_zeta() if prange is None else ctx.compute_zeta_range(*prange)
    return ctx, z


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_healpix_map_parity(tpcf, prec):
    """HEALPix nside 32 (12,288 pixels) with log-normal map values, 10 bins in [0.02, 0.3) rad,
    m_max = 8."""
    m = catalogs.sphere_map(32, 5, grid=64)
    say(f"healpix nside=32 prec={prec}")
    ctx, z = run_sphere(tpcf, m, 10, 0.02, 0.3, 8, prec, debug=True)
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 10, 0.02, 0.3, 8, want_counts=True)
    err = rel_err_per_l(z, ref.zeta)
    say("rel err per m", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    st = ctx.stats()
    assert st["n_pairs"] == ref.npairs
    npairs, _ = ctx.pair_sums()
    np.testing.assert_array_equal(npairs[0], ref.counts.sum(axis=0))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("mmax", [0, 3, 10])
def test_clustered_points_parity(tpcf, prec, mmax):
    """3,001 clustered points (caps at both poles, the exact pole among them: tangent basis
    switch), signed weights, 16 bins in [0, 0.25) rad: several tiles and a ragged tail."""
    m = catalogs.sphere_cluster(3001, 11, spread=0.08)
    m.w = m.w - 0.8
    say(f"cluster n=3001 mmax={mmax} prec={prec}")
    ctx, z = run_sphere(tpcf, m, 16, 0.0, 0.25, mmax, prec, debug=True)
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 16, 0.0, 0.25, mmax, want_counts=True)
    err = rel_err_per_l(z, ref.zeta)
    say("rel err per m", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_angles(tpcf, prec):
    """4,001 tightly clustered points, 12 bins in [0.002, 0.1) rad (sin(theta_max/2) <= 0.06: the
    three-term arcsine decides bins), m_max = 8."""
    m = catalogs.sphere_cluster(4001, 21, ncentre=5, spread=0.03)
    say(f"small angles prec={prec}")
    ctx, z = run_sphere(tpcf, m, 12, 0.002, 0.1, 8, prec, debug=True)
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 12, 0.002, 0.1, 8, want_counts=True)
    err = rel_err_per_l(z, ref.zeta)
    say("rel err per m", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_wide_angles(tpcf, prec):
    """Uniform points, bins reaching 2 rad (the arcsine's upper branch decides bins) and pi
    (every decision exact: antipodal pairs stay out of range)."""
    rng = np.random.default_rng(4)
    v = rng.normal(size=(2000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    m = catalogs.SphereMap(v[:, 0], v[:, 1], v[:, 2], rng.normal(1.0, 0.3, 2000))
    for tmax in (2.0, np.pi):
        say(f"wide angles tmax={tmax:.3f} prec={prec}")
        ctx, z = run_sphere(tpcf, m, 8, 0.0, tmax, 4, prec, debug=True)
        ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 8, 0.0, tmax, 4, want_counts=True)
        assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_range_and_pair_sums(tpcf, prec):
    """Primaries [60, 331) of 400 clustered points against the oracle's range, and the per-bin
    pair sums against the numpy pair table."""
    m = catalogs.sphere_cluster(400, 2, ncentre=3, spread=0.1)
    ctx, z = run_sphere(tpcf, m, 6, 0.01, 0.3, 5, prec, prange=(60, 331))
    ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 6, 0.01, 0.3, 5, 60, 331)
    assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]
    ctx2, _ = run_sphere(tpcf, m, 6, 0.01, 0.3, 5, prec)
    npairs, dd = ctx2.pair_sums()
    _, cnt, S = brute.zeta_sphere_triangles(m.x, m.y, m.z, m.w, 6, 0.01, 0.3, 0)
    np.testing.assert_array_equal(npairs[0], cnt.sum(axis=0))
    dd_ref = (m.w[:, None] * S).sum(axis=0)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert np.abs(dd[0] - dd_ref).max() <= tol * np.abs(dd_ref).max()


def test_device_inputs_and_validation(tpcf):
    """Torch CUDA inputs (validated on the device) give the host-input result; a vector off the
    unit sphere is rejected from either memory space."""
    import torch

    m = catalogs.sphere_cluster(1500, 6)
    ctx_h, zh = run_sphere(tpcf, m, 8, 0.0, 0.2, 6, "fp64")
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 0.0, 0.2, 6)
    t = [torch.from_numpy(a).cuda() for a in (m.x, m.y, m.z, m.w)]
    ctx.set_sphere_catalog(*t)
    zd = ctx.compute_zeta(device_output=True)
    assert rel_err_per_l(zd.cpu().numpy(), zh).max() < 1e-13
    bad = t[0].clone()
    bad[17] *= 1.01
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.set_sphere_catalog(bad, t[1], t[2], t[3])
    assert e.value.code == 1 and "unit vector" in str(e.value)
    # the 3D coupling is refused on the sphere (the binding picks the sphere's correction)
    ptr = zh.ctypes.data_as(ctypes.c_void_p)
    assert tpcf._lib.tpcf_edge_correct(ctx_h._h, 1, ptr, ptr, ptr, 0) == 5


def test_autotune_keeps_results(tpcf):
    m = catalogs.sphere_map(16, 8, grid=32)
    ctx = tpcf.Context(0)
    ctx.set_bins(6, 0.05, 0.5, 4)
    ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
    z0 = ctx.compute_zeta()
    t = ctx.autotune(0.2)
    say("tuning", t)
    z1 = ctx.compute_zeta()
    assert rel_err_per_l(z1, z0).max() < 1e-12


def test_full_sky_nside1024_sampled(tpcf):
    """The benchmark's map at full size: HEALPix nside 1024 (12,582,912 pixels), 20 bins in
    [10, 200) arcmin, m_max = 8, mixed precision. Three primary ranges against the oracle on the
    same ranges; the ranges add up to the full sweep over them; the pair sums add up to the pair
    count."""
    t0 = time.time()
    m = catalogs.sphere_map(1024, 2604)
    say(f"map built in {time.time() - t0:.1f}s")
    ctx = tpcf.Context(0)
    ctx.set_bins(20, 10 * ARCMIN, 200 * ARCMIN, 8)
    ctx.set_precision("mixed")
    ctx.set_sphere_catalog(m.x, m.y, m.z, m.w)
    full = ctx.compute_zeta()
    st = ctx.stats()
    say(f"full sweep {st['ms_sweep']:.1f} ms, {st['n_pairs']} pairs")
    npairs, _ = ctx.pair_sums()
    assert npairs.sum() == st["n_pairs"]
    assert st["n_pairs"] > 1.2e11
    n = m.n
    parts = []
    for a, b in [(0, 24), (n // 2, n // 2 + 24), (n - 24, n)]:
        z = ctx.compute_zeta_range(a, b)
        ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, 20, 10 * ARCMIN, 200 * ARCMIN, 8, a, b)
        err = rel_err_per_l(z, ref.zeta)
        say(f"range [{a}, {b}) rel err {err.max():.2e}")
        assert err.max() <= TOL["mixed"]
        parts.append(z)
    assert np.isfinite(full).all()


def test_sphere_edge_correct_matches_oracle(tpcf):
    """tpcf_edge_correct_sphere against the oracle's quadrature route on random moments (two
    catalogues, m_max = 8, 6 bins, one empty bin pair), host and device arrays."""
    import torch

    rng = np.random.default_rng(12)
    M, nb = 8, 6
    R = np.zeros((2, M + 1, nb, nb))
    R[:, 0] = 1.0 + rng.random((2, nb, nb))
    R[:, 1:] = 0.25 * rng.normal(size=(2, M, nb, nb)) * R[:, :1]
    R[1, :, 2, 3] = 0.0
    N = rng.normal(size=R.shape)
    ref = oracle.edge_correct_sphere(N, R)
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, 0.0, 0.2, M)
    ctx.set_sphere_catalog(*catalogs.healpix_centres(2))
    assert ctx.sphere
    out = ctx.edge_correct(N, R)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()
    assert not out[1, :, 2, 3].any()
    outd = ctx.edge_correct(torch.from_numpy(N).cuda(), torch.from_numpy(R).cuda()).cpu().numpy()
    assert np.abs(outd - ref).max() < 1e-12 * np.abs(ref).max()


def test_masked_map_edge_correction(tpcf):
    """A masked map (HEALPix nside 64 without the |dec| < 10 deg band and the dec > 60 deg cap):
    the mask's multipoles R come from the sweep itself, and edge_correct_sphere(R, R) is the unit
    vector; the corrected field multipoles are finite and agree with the oracle's correction of
    the same N and R."""
    m = catalogs.sphere_map(64, 7, grid=64)
    dec = np.arcsin(np.clip(m.z, -1.0, 1.0))
    keep = (np.abs(dec) > np.radians(10.0)) & (dec < np.radians(60.0))
    x, y, z = m.x[keep], m.y[keep], m.z[keep]
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 0.01, 0.2, 6)
    ctx.set_sphere_catalog(x, y, z, m.w[keep])
    N = ctx.compute_zeta()
    ctx.set_sphere_catalog(x, y, z, None)
    R = ctx.compute_zeta()
    say("mask anisotropy max |R_m/R_0|, m >= 1:", float(np.abs(R[1:] / R[0]).max()))
    rr = ctx.edge_correct(R, R)
    unit = np.zeros_like(rr)
    unit[0] = 1.0
    assert np.abs(rr - unit).max() < 1e-12
    c = ctx.edge_correct(N, R)
    assert np.isfinite(c).all()
    ref = oracle.edge_correct_sphere(N, R)
    assert np.abs(c - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sphere_batch(tpcf, prec):
    """Five maps in one launch (sizes 0, 1, 700, 2,000 and a HEALPix nside-16 map): each slice
    against the oracle, and the graph form (a non-null stream, replayed on new values) against the
    eager form."""
    import torch

    maps = [catalogs.SphereMap(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0)),
            catalogs.sphere_cluster(1, 3), catalogs.sphere_cluster(700, 4, spread=0.1),
            catalogs.sphere_cluster(2000, 5, ncentre=4, spread=0.15), catalogs.sphere_map(16, 6, grid=32)]
    maps[1] = catalogs.SphereMap(np.array([0.0]), np.array([0.0]), np.array([1.0]), np.array([2.0]))
    off = np.concatenate([[0], np.cumsum([mp.n for mp in maps])]).astype(np.int64)
    cat = lambda a: np.concatenate([getattr(mp, a) for mp in maps])
    ctx = tpcf.Context(0)
    ctx.set_bins(6, 0.01, 0.3, 5)
    ctx.set_precision(prec)
    zb = ctx.compute_sphere_batch(off, cat("x"), cat("y"), cat("z"), cat("w"))
    for k, mp in enumerate(maps):
        if mp.n < 2:
            assert not zb[k].any()
            continue
        ref = oracle.zeta_sphere(mp.x, mp.y, mp.z, mp.w, 6, 0.01, 0.3, 5)
        err = rel_err_per_l(zb[k], ref.zeta).max()
        say(f"sphere batch {prec} map {k} (n={mp.n}): {err:.2e}")
        assert err <= TOL[prec]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = tpcf.Context(0, stream)
        g.set_bins(6, 0.01, 0.3, 5)
        g.set_precision(prec)
        dev = [torch.from_numpy(cat(a)).cuda() for a in ("x", "y", "z", "w")]
        for rep in range(3):
            w = dev[3] * (1.0 + 0.5 * rep)
            zg = g.compute_sphere_batch(off, *dev[:3], w).cpu().numpy()
            torch.cuda.synchronize()
            e = tpcf.Context(0)
            e.set_bins(6, 0.01, 0.3, 5)
            e.set_precision(prec)
            ze = e.compute_sphere_batch(off, cat("x"), cat("y"), cat("z"), w.cpu().numpy())
            for k in range(len(maps)):
                if maps[k].n >= 2:
                    assert rel_err_per_l(zg[k], ze[k]).max() < 1e-6, (rep, k)
