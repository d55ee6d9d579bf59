"""The caller's allocator (tpcf_set_allocator through torch's caching allocator) and the device
byte cap (TPCF_MAX_DEVICE_BYTES): results unchanged against the oracle, the library's buffers
visible in torch's statistics while the context lives and returned when it closes, and calls
beyond the cap refused with TPCF_E_OUT_OF_MEMORY.
"""
import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_08855_amd as mod

    return mod


def test_torch_allocator(tpcf):
    """Single catalogue (mixed, debug rows on) and a graph-replayed batch, buffers from torch."""
    import torch

    cat = catalogs.uniform(8000, 200.0, 81)
    w = catalogs.gaussian_weights(cat.n, 82, 1.0, 0.3)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    say("torch allocator: single catalogue")
    ctx = tpcf.Context(0)
    ctx.use_torch_allocator()
    ctx.set_bins(10, 4.0, 40.0, 6)
    ctx.set_precision("mixed")
    ctx.set_debug(True)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
    z = ctx.compute_zeta()
    held = torch.cuda.memory_allocated() - base
    assert held >= 4 * 8 * cat.n  # at least the staged FP64 coordinates and weights
    ref = oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, 10, 4.0, 40.0, 6, want_counts=True)
    assert rel_err_per_l(z, ref.zeta).max() <= 1e-5
    np.testing.assert_array_equal(ctx.pair_counts(), ref.counts)
    D = ctx.degenerate()[0]
    Dref = oracle.degenerate(cat.x, cat.y, cat.z, w, cat.box, True, 10, 4.0, 40.0, 6)
    assert np.abs(D - Dref).max() <= 1e-10 * np.abs(Dref).max()

    say("torch allocator: batch replays")
    cats = [catalogs.uniform(n, 200.0, 90 + k) for k, n in enumerate((3000, 5000))]
    off = np.cumsum([0] + [c.n for c in cats]).astype(np.int64)
    x, y, zz = (np.concatenate([getattr(c, a) for c in cats]) for a in "xyz")
    refs = [oracle.zeta(c.x, c.y, c.z, None, c.box, True, 10, 4.0, 40.0, 6).zeta for c in cats]
    for _ in range(3):
        zb = ctx.compute_batch(off, x, y, zz, None, [200.0] * 2, [True] * 2)
        for k in range(len(cats)):
            assert rel_err_per_l(zb[k], refs[k]).max() <= 1e-5
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_device_byte_cap(tpcf, monkeypatch):
    """A cap below what the catalogue needs: TPCF_E_OUT_OF_MEMORY and a message naming the cap;
    without it the same context computes."""
    cat = catalogs.uniform(20000, 200.0, 83)
    ctx = tpcf.Context(0)
    ctx.set_bins(8, 4.0, 40.0, 4)
    monkeypatch.setenv("TPCF_MAX_DEVICE_BYTES", "100000")
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.set_catalog(cat.x, cat.y, cat.z, None, box=cat.box, periodic=True)
        ctx.compute_zeta()
    assert e.value.code == 3 and "TPCF_MAX_DEVICE_BYTES" in str(e.value)
    monkeypatch.delenv("TPCF_MAX_DEVICE_BYTES")
    ctx.set_catalog(cat.x, cat.y, cat.z, None, box=cat.box, periodic=True)
    z = ctx.compute_zeta()
    ref = oracle.zeta(cat.x, cat.y, cat.z, None, cat.box, True, 8, 4.0, 40.0, 4)
    assert rel_err_per_l(z, ref.zeta).max() <= 1e-10
