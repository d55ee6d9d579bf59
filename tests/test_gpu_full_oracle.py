"""The whole 1,000,000-point log-normal catalogue (periodic cube of side 1000, weights
1 + 0.1 N(0,1), 20 bins over [10, 200), l_max = 10; the benchmark's catalogue) against the FP64
oracle's zeta over every primary, stored in tests/golden/lognormal1e6_oracle.txt by
tests/golden/make_lognormal1e6_oracle.py (which calls only the input generator and the oracle).

The catalogue is regenerated here and must hash to the stored sha256: a mismatch fails the test
(the generator changed, so the stored values no longer apply). Then, element by element over
(l, r1, r2), |zeta - zeta_oracle| / max |zeta_oracle_l| stays within 1e-10 on the FP64 path and
1e-5 on the mixed path, and the ordered pair total and the pair count of every bin are exact.
"""
import importlib.util
import os

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _fixture_module():
    spec = importlib.util.spec_from_file_location(
        "make_lognormal1e6_oracle", os.path.join(ROOT, "tests", "golden", "make_lognormal1e6_oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


FX = _fixture_module()


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available()
    import paper_2604_08855_amd as mod

    return mod


@pytest.fixture(scope="module")
def gold():
    return FX.read()


@pytest.fixture(scope="module")
def catalogue(gold):
    say("generating the 1e6-point log-normal catalogue")
    cat, w = FX.catalogue()
    digest = FX.catalogue_hash(cat, w)
    assert digest == gold["sha256"], f"catalogue hash {digest} differs from the stored oracle's {gold['sha256']}"
    return cat, w


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_catalogue_matches_oracle(tpcf, catalogue, gold, prec):
    cat, w = catalogue
    ctx = tpcf.Context(0)
    ctx.set_bins(FX.NB, FX.RMIN, FX.RMAX, FX.LMAX)
    ctx.set_precision(prec)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=FX.BOX, periodic=True)
    say(f"full catalogue, prec={prec}")
    z = ctx.compute_zeta()
    st = ctx.stats()
    npairs, _ = ctx.pair_sums()
    assert st["n_pairs"] == gold["npairs"]
    np.testing.assert_array_equal(npairs[0], gold["bin_pairs"])
    ref = gold["zeta"]
    scale = np.abs(ref).reshape(FX.LMAX + 1, -1).max(axis=1)
    err = np.abs(z - ref) / scale[:, None, None]
    l, b1, b2 = np.unravel_index(int(np.argmax(err)), err.shape)
    say(f"{prec}: max error per l {err.reshape(FX.LMAX + 1, -1).max(axis=1)}; worst at (l={l}, r1={b1}, r2={b2})")
    assert err.max() <= TOL[prec]
