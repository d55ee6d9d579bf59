"""GPU parity: the HIP path against the FP64 oracle on identical seeded inputs.

Bars (floating point): FP64 path max|zeta_l - oracle_l| <= 1e-10 * max|oracle_l| per l; mixed
path <= 1e-5 * max|oracle_l| per l. Integer per-primary per-bin pair counts are bit-exact.
"""
import math

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


def run_gpu(tpcf, cat, w, nb, rmin, rmax, lmax, prec, debug=False, tuning=None, prange=None):
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, lmax)
    ctx.set_precision(prec)
    if tuning:
        ctx.set_tuning(*tuning)
    ctx.set_debug(debug)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=cat.periodic)
    z = ctx.compute_zeta() if prange is None else ctx.compute_zeta_range(*prange)
    return ctx, z


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_config_full_parity(tpcf, prec):
    """10,000 uniform points, periodic box 250, 10 bins [5, 50), l_max = 4."""
    cat = catalogs.uniform(10000, 250.0, 0)
    say(f"small config n=10000 prec={prec}")
    ctx, z = run_gpu(tpcf, cat, None, 10, 5.0, 50.0, 4, prec, debug=True)
    ref = oracle.zeta_catalog(cat, 10, 5.0, 50.0, 4, want_counts=True)
    err = rel_err_per_l(z, ref.zeta)
    say("rel err per l", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    st = ctx.stats()
    assert st["n_pairs"] == ref.npairs
    assert st["n_candidates"] >= st["n_pairs"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
def test_weighted_lmax10_parity(tpcf, prec, periodic):
    """Several tiles and a ragged tail: 3,001 points, 20 bins, l_max = 10, signed weights."""
    cat = catalogs.uniform(3001, 160.0, 7)
    cat.periodic = periodic
    w = catalogs.gaussian_weights(cat.n, 8, 0.3, 1.0)
    say(f"weighted lmax10 periodic={periodic} prec={prec}")
    ctx, z = run_gpu(tpcf, cat, w, 20, 3.0, 45.0, 10, prec, debug=True)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, periodic, 20, 3.0, 45.0, 10, want_counts=True)
    err = rel_err_per_l(z, ref.zeta)
    say("rel err per l", err)
    assert err.max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_alm_against_oracle(tpcf, prec):
    """Normalised a_lm of every primary and bin against the oracle.

    The kernel accumulates Chebyshev moments sum_j w_j T_k(z_j) (x_j - i y_j)^m, coherent sums
    of size up to sum_j |w_j|, and forms a_lm = sum_k E_lmk M_{m,k} afterwards. Its rounding is
    therefore bounded relative to sum_{j in bin} |w_j| times sum_k |E_lmk|, and
    sum_k |E_lmk| = N_lm (l+m)! / (2^m m! (l-m)!) because every Chebyshev coefficient of
    d^m P_l / dz^m is non-negative (their sum is the derivative at z = 1). The bar:
    |a_gpu - a_oracle| <= tol * sum_{j in bin} |w_j| * N_lm (l+m)! / (2^m m! (l-m)!).
    """
    cat = catalogs.uniform(700, 60.0, 3)
    w = catalogs.gaussian_weights(cat.n, 4)
    L, nb = 10, 5
    say(f"a_lm parity prec={prec}")
    ctx, _ = run_gpu(tpcf, cat, w, nb, 2.0, 20.0, L, prec, debug=True)
    a = ctx.alm()  # [n, nb, l, m]
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, nb, 2.0, 20.0, L, want_alm=True).alm
    # coherent scale sum_{j in bin} |w_j| from the oracle's own l = 0 shell of |w|
    absw = oracle.zeta(cat.x, cat.y, cat.z, np.abs(w), cat.box, True, nb, 2.0, 20.0, 0, want_alm=True).alm
    wsum = np.abs(absw[:, :, 0]) * math.sqrt(4 * math.pi)
    tol = 1e-12 if prec == "fp64" else 2e-5
    worst = 0.0
    for l in range(L + 1):
        for m in range(l + 1):
            nlm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            g1 = math.factorial(l + m) / (2**m * math.factorial(m) * math.factorial(l - m))
            bound = wsum * nlm * g1 + 1e-300
            err = np.abs(a[:, :, l, m] - ref[:, :, l * l + l + m]) / bound
            worst = max(worst, float(err.max()))
    say("worst a_lm error / coherent scale", worst)
    assert worst < tol


@pytest.mark.parametrize("lmax", list(range(0, 11)))
def test_every_lmax(tpcf, lmax):
    cat = catalogs.uniform(900, 80.0, 20 + lmax)
    w = catalogs.gaussian_weights(cat.n, 40 + lmax)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 7, 2.0, 30.0, lmax).zeta
    for prec in ("fp64", "mixed"):
        _, z = run_gpu(tpcf, cat, w, 7, 2.0, 30.0, lmax, prec)
        assert rel_err_per_l(z, ref).max() <= TOL[prec], (lmax, prec)


@pytest.mark.parametrize("nb", [1, 2, 16, 17, 32])
def test_bin_counts(tpcf, nb):
    cat = catalogs.uniform(1200, 70.0, 30 + nb)
    ref = oracle.zeta(cat.x, cat.y, cat.z, None, cat.box, True, nb, 1.0, 30.0, 3, want_counts=True)
    for prec in ("fp64", "mixed"):
        ctx, z = run_gpu(tpcf, cat, None, nb, 1.0, 30.0, 3, prec, debug=True)
        assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


def test_degenerate_inputs(tpcf):
    for n in (0, 1):
        cat = catalogs.uniform(n, 50.0, 1)
        for prec in ("fp64", "mixed"):
            _, z = run_gpu(tpcf, cat, None, 4, 1.0, 10.0, 4, prec)
            assert z.shape == (5, 4, 4) and not z.any()
    # coincident points with r_min = 0: no direction, no pair
    c = catalogs.Catalog(np.array([5.0, 5.0]), np.array([5.0, 5.0]), np.array([5.0, 5.0]), np.ones(2), 50.0, True)
    ctx, z = run_gpu(tpcf, c, None, 4, 0.0, 10.0, 2, "fp64", debug=True)
    assert not z.any() and ctx.stats()["n_pairs"] == 0


def test_exact_bin_edges(tpcf):
    box, K = 256.0, 27
    s = box / 2**K
    x0 = 100.0 + 0.5 * s
    xs = np.array([x0, x0 + 16.0, x0 + 16.0 - s, x0 + 64.0, x0 + 8.0, x0 - 24.0, x0 - 24.0 + s])
    ys = np.full(xs.shape, 50.0 + 0.5 * s)
    c = catalogs.Catalog(xs, ys, ys, np.ones(len(xs)), box, True)
    ref = oracle.zeta(xs, ys, ys, None, box, True, 7, 8.0, 64.0, 2, want_counts=True)
    for prec in ("fp64", "mixed"):
        ctx, z = run_gpu(tpcf, c, None, 7, 8.0, 64.0, 2, prec, debug=True)
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
        assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec]


def test_primary_ranges_add_up(tpcf):
    cat = catalogs.uniform(2500, 100.0, 51)
    w = catalogs.gaussian_weights(cat.n, 52)
    args = (w, 6, 2.0, 30.0, 6, "fp64")
    _, full = run_gpu(tpcf, cat, *args)
    _, a = run_gpu(tpcf, cat, *args, prange=(0, 1111))
    _, b = run_gpu(tpcf, cat, *args, prange=(1111, 2500))
    assert rel_err_per_l(a + b, full).max() < 1e-12
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 6, 2.0, 30.0, 6, 0, 1111).zeta
    assert rel_err_per_l(a, ref).max() < 1e-10


@pytest.mark.parametrize("tuning", [(5.0, 1, 64), (80.0, 3, 128), (2.0, 8, 4096)])
def test_tuning_does_not_change_results(tpcf, tuning):
    """Small cells, large cells, a tiny scratch area (forces shells flushed in several chunks)."""
    cat = catalogs.lognormal(4000, 200.0, 9, grid=32)
    w = catalogs.gaussian_weights(cat.n, 10)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 12, 5.0, 60.0, 8, want_counts=True)
    for prec in ("fp64", "mixed"):
        ctx, z = run_gpu(tpcf, cat, w, 12, 5.0, 60.0, 8, prec, debug=True, tuning=tuning)
        assert rel_err_per_l(z, ref.zeta).max() <= TOL[prec], (tuning, prec)
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
def test_pair_sums_match_oracle(tpcf, prec, periodic):
    """Two-point by-product: ordered pairs per bin (exact) and sum of w_p w_j per bin, for the
    whole catalogue and for a primary range."""
    cat = catalogs.lognormal(5000, 150.0, 71, grid=32, periodic=periodic)
    w = catalogs.gaussian_weights(cat.n, 72, 1.0, 0.5)
    tol = 1e-12 if prec == "fp64" else 2e-6
    ctx, _ = run_gpu(tpcf, cat, w, 9, 3.0, 45.0, 5, prec)
    for rng in (None, (700, 2345)):
        if rng is not None:
            ctx.compute_zeta_range(*rng)
        npairs, dd = ctx.pair_sums()
        assert npairs.shape == (1, 9)
        b0, b1 = rng if rng else (0, cat.n)
        rn, rdd = oracle.pair_sums(cat.x, cat.y, cat.z, w, cat.box, periodic, 9, 3.0, 45.0, b0, b1)
        np.testing.assert_array_equal(npairs[0], rn)
        err = np.max(np.abs(dd[0] - rdd)) / np.max(np.abs(rdd))
        say(f"pair sums {prec} periodic={periodic} range={rng}: dd rel err {err:.2e}")
        assert err <= tol


def test_edge_correct_matches_oracle_on_random_multipoles(tpcf):
    """The coupling-matrix solve against the oracle's quadrature route, l_max = 10, two
    catalogues, host and device arrays, a bin pair without randoms."""
    import torch

    rng = np.random.default_rng(81)
    L, nb = 10, 5
    R = rng.normal(0.0, 0.15, (2, L + 1, nb, nb))
    R[:, 0] = rng.uniform(0.5, 2.0, (2, nb, nb))
    R *= R[:, :1]  # f_l = R_l / R_0 stays small
    R[1, :, 2, 3] = 0.0
    N = rng.normal(size=(2, L + 1, nb, nb))
    ref = oracle.edge_correct(N, R)
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, 1.0, 10.0, L)
    z = ctx.edge_correct(N, R)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert not z[1, :, 2, 3].any()
    zd = ctx.edge_correct(torch.from_numpy(N).cuda(), torch.from_numpy(R).cuda())
    assert zd.is_cuda
    assert np.max(np.abs(zd.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_edge_corrected_data_minus_randoms(tpcf):
    """End to end: N from the data-minus-randoms field, R from the randoms alone (weight
    +N_d/N_r), both on the GPU (FP64), corrected on the GPU; against the oracle's N and R
    corrected by the oracle."""
    cat = catalogs.data_minus_randoms(1500, 4500, 120.0, 91, 92, grid=32)
    nd = 1500
    nb, rmin, rmax, L = 6, 4.0, 30.0, 6
    rand = slice(nd, cat.n)
    wr = -cat.w[rand]
    ctx = tpcf.Context(0)
    ctx.set_bins(nb, rmin, rmax, L)
    ctx.set_precision("fp64")
    ctx.set_catalog(cat.x, cat.y, cat.z, cat.w, box=cat.box, periodic=False)
    Ng = ctx.compute_zeta()
    ctx.set_catalog(cat.x[rand], cat.y[rand], cat.z[rand], wr, box=cat.box, periodic=False)
    Rg = ctx.compute_zeta()
    zg = ctx.edge_correct(Ng, Rg)
    No = oracle.zeta(cat.x, cat.y, cat.z, cat.w, cat.box, False, nb, rmin, rmax, L).zeta
    Ro = oracle.zeta(cat.x[rand], cat.y[rand], cat.z[rand], wr, cat.box, False, nb, rmin, rmax, L).zeta
    zo = oracle.edge_correct(No, Ro)
    assert Ro[0].min() > 0
    err = rel_err_per_l(zg, zo)
    say("edge-corrected rel err per l", err)
    assert err.max() <= 1e-9


def test_settings_changed_between_calls_rebuild_the_grid(tpcf):
    """One context, one catalogue: new tuning, then new bins, between compute calls. Every call
    must match the oracle for the settings in force (the cell grid is rebuilt when its
    geometry changes)."""
    cat = catalogs.lognormal(5000, 200.0, 41, grid=32)
    w = catalogs.gaussian_weights(cat.n, 42)
    ctx = tpcf.Context(0)
    ctx.set_precision("fp64")
    ctx.set_debug(True)
    ctx.set_bins(8, 4.0, 40.0, 5)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 8, 4.0, 40.0, 5, want_counts=True)
    for ppc in (8.0, 2.0, 24.0):
        ctx.set_tuning(ppc, 0, 0)
        z = ctx.compute_zeta()
        say(f"ppc={ppc}", rel_err_per_l(z, ref.zeta).max())
        assert rel_err_per_l(z, ref.zeta).max() <= TOL["fp64"]
        np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    ctx.set_bins(6, 2.0, 60.0, 4)
    ref2 = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 6, 2.0, 60.0, 4, want_counts=True)
    z = ctx.compute_zeta()
    assert rel_err_per_l(z, ref2.zeta).max() <= TOL["fp64"]
    np.testing.assert_array_equal(ctx.pair_counts(), ref2.counts)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_keeps_results(tpcf, prec):
    """The autotuner picks a configuration from its candidate set; results after it still match
    the oracle, with exact pair counts. Stats of the last compute call are kept; its debug output
    is dropped."""
    cat = catalogs.lognormal(6000, 200.0, 31, grid=32)
    w = catalogs.gaussian_weights(cat.n, 32)
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 10, 4.0, 50.0, 6, want_counts=True)
    ctx, z0 = run_gpu(tpcf, cat, w, 10, 4.0, 50.0, 6, prec, debug=True)
    counts0 = ctx.pair_counts()
    st0 = ctx.stats()
    t = ctx.autotune(0.25)
    say("autotune", t)
    assert t["points_per_cell"] in (3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0)
    assert t["waves_per_cu"] in (12, 8)
    assert t["candidates"] == 20
    assert t["scratch_blocks"] in (512, 1024, 2048)
    assert 0.0 < t["ms_best"] <= t["ms_default"]
    assert ctx.stats() == st0
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.pair_counts()
    assert e.value.code == 2
    np.testing.assert_array_equal(counts0, ref.counts)
    z1 = ctx.compute_zeta()
    assert rel_err_per_l(z1, ref.zeta).max() <= TOL[prec]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    assert rel_err_per_l(z0, ref.zeta).max() <= TOL[prec]


def test_device_tensors_in_and_out(tpcf):
    import torch

    cat = catalogs.uniform(2000, 90.0, 61)
    w = catalogs.gaussian_weights(cat.n, 62)
    t = [torch.from_numpy(a).cuda() for a in (cat.x, cat.y, cat.z, w)]
    z = tpcf.zeta(*t, box=cat.box, periodic=True, rmin=2.0, rmax=25.0, nbins=6, lmax=5,
                  precision="mixed")
    assert z.is_cuda and z.dtype == torch.float64
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 6, 2.0, 25.0, 5).zeta
    assert rel_err_per_l(z.cpu().numpy(), ref).max() <= 1e-5
    # invalid device data is reported, not computed
    bad = t[0].clone()
    bad[17] = float("nan")
    with pytest.raises(tpcf.TpcfError) as e:
        tpcf.zeta(bad, t[1], t[2], box=cat.box, periodic=True, rmin=2.0, rmax=25.0, nbins=6, lmax=5)
    assert e.value.code == 1


@pytest.mark.parametrize("where", ["host", "device"])
def test_fp32_inputs(tpcf, where):
    """tpcf_set_catalog_f32 / tpcf_set_sphere_catalog_f32 (numpy float32 on the host, torch float32
    on the device): the same result as the oracle on the values widened to FP64."""
    import torch

    cat = catalogs.uniform(4000, 150.0, 71)
    w = catalogs.gaussian_weights(cat.n, 72, 0.5, 1.0)
    f = [np.minimum(a.astype(np.float32), np.nextafter(np.float32(150.0), np.float32(0))) for a in (cat.x, cat.y, cat.z)]
    wf = w.astype(np.float32)
    say(f"fp32 inputs on the {where}")
    args = [torch.from_numpy(a).cuda() for a in (*f, wf)] if where == "device" else [*f, wf]
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 4.0, 30.0, 4)
    ctx.set_precision("fp64")
    ctx.set_debug(True)
    ctx.set_catalog(*args, box=150.0, periodic=True)
    z = ctx.compute_zeta()
    x64, y64, z64, w64 = (a.astype(np.float64) for a in (*f, wf))
    ref = oracle.zeta(x64, y64, z64, w64, 150.0, True, 8, 4.0, 30.0, 4, want_counts=True)
    assert rel_err_per_l(z, ref.zeta).max() <= TOL["fp64"]
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)

    m = catalogs.sphere_map(16, 73, grid=32)
    u = [a.astype(np.float32) for a in (m.x, m.y, m.z, m.w)]
    args = [torch.from_numpy(a).cuda() for a in u] if where == "device" else u
    ctx = tpcf.Context(0)
    ctx.set_bins(6, 0.05, 0.5, 5)
    ctx.set_precision("fp64")
    ctx.set_sphere_catalog(*args)
    zs = ctx.compute_zeta()
    u64 = [a.astype(np.float64) for a in u]
    ref = oracle.zeta_sphere(*u64, 6, 0.05, 0.5, 5)
    assert rel_err_per_l(zs, ref.zeta).max() <= TOL["fp64"]
