"""Parity at the benchmark's full size (1e6 log-normal points, L = 1000, 20 bins [10, 200),
l_max = 10) and at a non-periodic data-minus-randoms configuration.

The oracle cannot do the whole catalogue in seconds, so it checks a random sample of primaries
(every secondary of each) through tpcf_compute_zeta_range, in the same launch configuration the
benchmark uses; the full-catalogue result is checked through properties that hold at any size
(symmetry, positive semi-definiteness for positive weights, mixed vs FP64 agreement, and the
total pair count equal to the sum of exact per-primary counts)."""
import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu
NB, RMIN, RMAX, L = 20, 10.0, 200.0, 10


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available()
    import paper_2604_08855_amd as mod

    return mod


@pytest.fixture(scope="module")
def c3():
    cat = catalogs.lognormal(1_000_000, 1000.0, 0, grid=256)
    cat.w = catalogs.gaussian_weights(cat.n, 10**6, 1.0, 0.1)
    return cat


def ctx_for(tpcf, cat, prec, debug=False):
    ctx = tpcf.Context(0)
    ctx.set_bins(NB, RMIN, RMAX, L)
    ctx.set_precision(prec)
    ctx.set_debug(debug)
    ctx.set_catalog(cat.x, cat.y, cat.z, cat.w, box=cat.box, periodic=cat.periodic)
    return ctx


def test_full_size_properties(tpcf, c3):
    say("full size: mixed and fp64 over 1e6 points")
    cm = ctx_for(tpcf, c3, "mixed")
    zm = cm.compute_zeta()
    sm = cm.stats()
    cf = ctx_for(tpcf, c3, "fp64")
    zf = cf.compute_zeta()
    sf = cf.stats()
    say("pairs", sm["n_pairs"], "sweep ms mixed", sm["ms_sweep"], "fp64", sf["ms_sweep"])
    assert sm["n_pairs"] == sf["n_pairs"]
    err = rel_err_per_l(zm, zf)
    say("mixed vs fp64 per l", err)
    assert err.max() <= 1e-5
    for l in range(L + 1):
        np.testing.assert_allclose(zf[l], zf[l].T, rtol=0, atol=1e-12 * np.abs(zf[l]).max())
        ev = np.linalg.eigvalsh(0.5 * (zf[l] + zf[l].T))
        assert ev.min() >= -1e-10 * ev.max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sampled_primaries_against_oracle(tpcf, c3, prec):
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(c3.n, size=24, replace=False))
    ctx = ctx_for(tpcf, c3, prec, debug=True)
    z = np.zeros((L + 1, NB, NB))
    ref = np.zeros_like(z)
    for p in sample:
        z += ctx.compute_zeta_range(int(p), int(p) + 1)
        counts = ctx.pair_counts()[p]
        r = oracle.zeta(c3.x, c3.y, c3.z, c3.w, c3.box, True, NB, RMIN, RMAX, L, int(p), int(p) + 1,
                        want_counts=True)
        ref += r.zeta
        np.testing.assert_array_equal(counts, r.counts[0])
    err = rel_err_per_l(z, ref)
    say(prec, "sampled-primary rel err per l", err)
    assert err.max() <= (1e-10 if prec == "fp64" else 1e-5)


def test_total_pairs_equal_sum_of_exact_counts(tpcf, c3):
    ctx = ctx_for(tpcf, c3, "mixed", debug=True)
    ctx.compute_zeta()
    counts = ctx.pair_counts()
    assert counts.sum() == ctx.stats()["n_pairs"]
    assert counts.min() >= 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_data_minus_randoms_nonperiodic(tpcf, prec):
    """Non-periodic cube, clustered data (w = 1) plus uniform randoms (w = -N_d/N_r), the density
    of the 4e6 + 1.6e7 point configuration at a fifth of its volume."""
    box = 2000.0 / 5 ** (1 / 3)
    cat = catalogs.data_minus_randoms(800_000, 3_200_000, box, 5, 6, grid=128)
    rng = np.random.default_rng(7)
    # primaries near the walls and in the bulk, data and randoms
    near = np.where(np.min(np.stack([cat.x, cat.y, cat.z, box - cat.x, box - cat.y, box - cat.z]), 0) < 30.0)[0]
    sample = np.sort(np.concatenate([rng.choice(near, 8, replace=False),
                                     rng.choice(cat.n, 8, replace=False)]))
    ctx = ctx_for(tpcf, cat, prec, debug=True)
    z = np.zeros((L + 1, NB, NB))
    ref = np.zeros_like(z)
    for p in sample:
        z += ctx.compute_zeta_range(int(p), int(p) + 1)
        counts = ctx.pair_counts()[p]
        r = oracle.zeta(cat.x, cat.y, cat.z, cat.w, box, False, NB, RMIN, RMAX, L, int(p), int(p) + 1,
                        want_counts=True)
        ref += r.zeta
        np.testing.assert_array_equal(counts, r.counts[0])
    err = rel_err_per_l(z, ref)
    say(prec, "non-periodic sampled rel err", err)
    assert err.max() <= (1e-10 if prec == "fp64" else 1e-5)


def test_data_minus_randoms_mixed_vs_fp64_full():
    """The whole data-minus-randoms catalogue at a fifth of the 4e6 + 1.6e7 configuration's volume
    (same density, non-periodic): the mixed zeta against the FP64 zeta element by element over
    (l, r1, r2), relative to max |zeta_l|, within 1e-5, despite the cancellation between the data
    (w = 1) and the randoms (w = -1/4); pair counts identical."""
    import paper_2604_08855_amd as tpcf

    box = 2000.0 / 5 ** (1 / 3)
    cat = catalogs.data_minus_randoms(800_000, 3_200_000, box, 5, 6, grid=128)
    out = {}
    for prec in ("fp64", "mixed"):
        say(f"data minus randoms, full, {prec}")
        ctx = ctx_for(tpcf, cat, prec)
        out[prec] = (ctx.compute_zeta(), ctx.stats()["n_pairs"])
    assert out["fp64"][1] == out["mixed"][1]
    err = rel_err_per_l(out["mixed"][0], out["fp64"][0])
    say("mixed vs fp64 per l", err)
    assert err.max() <= 1e-5
