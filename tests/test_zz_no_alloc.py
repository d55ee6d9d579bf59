"""tpcf_compute_batch_noalloc, the batch entry point for callers that cannot allocate device memory:
its output matches tpcf_compute_batch's on the same inputs (bit for bit in the deterministic form,
within the oracle bars otherwise, exact pair counts either way) on two calls in a row, the second
with a smaller batch, while the caller's allocator of its context (one that always fails) is never
called. Batches too large for the static array are refused with a clear error, and the context
stays usable.
"""
import ctypes

import numpy as np
import pytest

import catalogs
import oracle
from tests.gpu_util import rel_err_per_l, say
from tests.test_gpu_batch import concat, make_batch

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
NB, RMIN, RMAX, L = 8, 3.0, 30.0, 6

_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


@pytest.fixture(scope="module")
def tpcf():
    import torch

    assert torch.cuda.is_available()
    import paper_2604_08855_amd as mod

    return mod


def refusing_allocator(tpcf, ctx):
    """Installs an allocator that counts its calls and always fails; returns the counter."""
    calls = [0]

    @_ALLOC
    def alloc(nbytes, user):
        calls[0] += 1
        return None

    @_FREE
    def free(ptr, user):
        calls[0] += 1

    ctx._keep_alloc = (alloc, free)
    assert tpcf._lib.tpcf_set_allocator(ctx._h, ctypes.cast(alloc, ctypes.c_void_p),
                                        ctypes.cast(free, ctypes.c_void_p), None) == 0
    return calls


def small_batch(seed):
    """Three catalogues, 0 to 1500 points: smaller in total than make_batch's 7301."""
    specs = [(1500, 110.0, True), (0, 100.0, False), (900, 80.0, False)]
    cats = []
    for k, (n, box, per) in enumerate(specs):
        c = catalogs.uniform(n, box, seed + k)
        c.periodic = per
        c.w = catalogs.gaussian_weights(n, 300 + seed + k)
        cats.append(c)
    return cats


def make_ctx(tpcf, prec, det):
    ctx = tpcf.Context(0)
    ctx.set_bins(NB, RMIN, RMAX, L)
    ctx.set_precision(prec)
    ctx.set_deterministic(det)
    return ctx


@pytest.mark.parametrize("det", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_compute_batch(tpcf, prec, det):
    import torch

    ref_ctx = make_ctx(tpcf, prec, det)
    na_ctx = make_ctx(tpcf, prec, det)
    calls = refusing_allocator(tpcf, na_ctx)
    for label, cats in (("7301 points", make_batch(31)), ("2400 points", small_batch(41))):
        off, x, y, z, w = concat(cats)
        boxes, pers = [c.box for c in cats], [c.periodic for c in cats]
        say(f"noalloc prec={prec} det={det}: batch of {len(cats)} catalogues, {label}")
        dev = [torch.from_numpy(a).cuda() for a in (x, y, z, w)]
        out = torch.full((len(cats), L + 1, NB, NB), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        na_ctx.compute_batch_noalloc(off, *dev, boxes, pers, out=out)
        got = out.cpu().numpy()
        assert calls[0] == 0, "the no-alloc entry point called the context's allocator"
        na_stats = na_ctx.stats()
        ref = ref_ctx.compute_batch(off, x, y, z, w, boxes, pers)
        assert na_stats["n_pairs"] == ref_ctx.stats()["n_pairs"]
        say("waves", na_stats["waves"], "vs", ref_ctx.stats()["waves"], "pairs", na_stats["n_pairs"])
        if det:
            assert np.array_equal(got, ref)
        for k, c in enumerate(cats):
            if not np.abs(ref[k]).max() > 0.0:
                assert not got[k].any()
                continue
            assert rel_err_per_l(got[k], ref[k]).max() <= TOL[prec]
            o = oracle.zeta(c.x, c.y, c.z, c.w, c.box, c.periodic, NB, RMIN, RMAX, L).zeta
            assert rel_err_per_l(got[k], o).max() <= TOL[prec]
        # the two-point sums of a no-alloc call lived in the static array
        with pytest.raises(tpcf.TpcfError):
            na_ctx.pair_sums()
    # the refusing allocator is really the context's: the allocating entry point fails on it
    off, x, y, z, w = concat(small_batch(41))
    with pytest.raises(tpcf.TpcfError) as e:
        na_ctx.compute_batch(off, x, y, z, w, [1.0e3] * 3, [0] * 3)
    assert "OUT_OF_MEMORY" in str(e.value) and calls[0] > 0


def test_noalloc_keeps_the_context(tpcf):
    """A regular catalogue set on the context survives a no-alloc call in between."""
    import torch

    cat = catalogs.uniform(3000, 100.0, 51)
    w = catalogs.gaussian_weights(cat.n, 52)
    ctx = make_ctx(tpcf, "fp64", False)
    ctx.set_catalog(cat.x, cat.y, cat.z, w, box=cat.box, periodic=True)
    z1 = ctx.compute_zeta()
    cats = small_batch(61)
    off, x, y, z, wb = concat(cats)
    out = torch.empty((len(cats), L + 1, NB, NB), dtype=torch.float64, device="cuda")
    ctx.compute_batch_noalloc(off, *[torch.from_numpy(a).cuda() for a in (x, y, z, wb)],
                              [c.box for c in cats], [c.periodic for c in cats], out=out)
    z2 = ctx.compute_zeta()
    assert rel_err_per_l(z2, z1).max() <= TOL["fp64"]
    assert ctx.stats()["n_pairs"] == oracle.zeta(cat.x, cat.y, cat.z, w, cat.box, True, NB, RMIN, RMAX, L).npairs


def test_noalloc_refuses_oversized_batch(tpcf):
    """Four million points do not fit in the static array: refused with OUT_OF_MEMORY and a
    message naming the array; the same context then computes a small batch correctly."""
    import torch

    n = 4_000_000
    g = torch.Generator(device="cuda").manual_seed(7)
    xyz = [torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 1000.0 for _ in range(3)]
    ctx = make_ctx(tpcf, "mixed", False)
    out = torch.empty((1, L + 1, NB, NB), dtype=torch.float64, device="cuda")
    say("noalloc: 4e6 points (refused)")
    with pytest.raises(tpcf.TpcfError) as e:
        ctx.compute_batch_noalloc(np.array([0, n]), *xyz, None, [1000.0], [1], out=out)
    assert "OUT_OF_MEMORY" in str(e.value) and "static scratch" in str(e.value)
    say(str(e.value))
    cats = small_batch(71)
    off, x, y, z, w = concat(cats)
    out = torch.empty((len(cats), L + 1, NB, NB), dtype=torch.float64, device="cuda")
    ctx.compute_batch_noalloc(off, *[torch.from_numpy(a).cuda() for a in (x, y, z, w)],
                              [c.box for c in cats], [c.periodic for c in cats], out=out)
    got = out.cpu().numpy()
    for k, c in enumerate(cats):
        o = oracle.zeta(c.x, c.y, c.z, c.w, c.box, c.periodic, NB, RMIN, RMAX, L).zeta
        if np.abs(o).max() > 0:
            assert rel_err_per_l(got[k], o).max() <= TOL["mixed"]
