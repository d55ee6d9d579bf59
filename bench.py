"""Benchmark: primary-secondary pairs per second of the 3PCF multipole hot path on one MI355X.

Workload (the precision form of the paper's fast estimator at scale): 1,000,000 points
Poisson-sampled from a log-normal density field (Gaussian field, P(k) ~ k^-1.5, sigma_lnrho = 1,
256^3 grid) in a periodic cube of side 1000 Mpc/h, weights 1 + 0.1 N(0,1), 20 linear bins over
[10, 200) Mpc/h, l_max = 10, mixed precision (FP32 sweep with Kahan shells, split-BF16 MFMA
contraction, FP64 global reduction).

One step = the whole hot path on device-resident inputs: lattice snap + cell-grid build, pair
sweep with the a_lm shells, contraction into zeta_l(r1, r2). The same catalogue is also timed on
the FP64 path (FP64 sweep and FP64 MFMA contraction), and the mixed result is compared with it.

Before the warmup, the library's autotuner picks the grid density and wave count on a 5% sample of
primaries (outside the timed steps; --no-autotune keeps the defaults).

Prints one JSON line. Options: --steps K --warmup W --gpus N (only 1 is supported)
--cpu-seconds S (target wall time of the oracle sample; 0 skips the CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NB, RMIN, RMAX, LMAX, BOX, N = 20, 10.0, 200.0, 10, 1000.0, 1_000_000
# HBM counters of the sweep kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated on a plain copy)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_lognormal1e6_hbm_traffic.md")
SPHERE_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_sphere_nside1024_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_08855_amd", "csrc", f) for f in ("sweep.hip", "tpcf_internal.h")]
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32, published (counts packed FP32 instructions)
# The same chip without packed FP32 (which the library's build leaves off): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops per FMA x 2.4 GHz.
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
F_PAIR = 4 * (LMAX + 1) ** 2  # algorithmic flops per in-range pair (2 to generate + 2 to add)
F_PRIM = 2 * NB * NB * (LMAX + 1) ** 2  # algorithmic flops per primary for the contraction


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PHASE_ALIGNED = -1  # --phase-aligned: -1 by neighbourhood size, 0 off, 1 on
DETERMINISTIC = False  # --deterministic: fixed tiles and a fixed-order reduction


def make_ctx(tpcf, stream):
    """A library context on device 0 and `stream`, with the run's phase-alignment and
    deterministic settings."""
    ctx = tpcf.Context(0, stream)
    ctx.set_phase_aligned(PHASE_ALIGNED)
    ctx.set_deterministic(DETERMINISTIC)
    return ctx


def make_catalog():
    import catalogs

    t0 = time.time()
    cat = catalogs.lognormal(N, BOX, 0, grid=256)
    w = catalogs.gaussian_weights(N, 10**6, 1.0, 0.1)
    log(f"[bench] catalogue generated in {time.time() - t0:.1f}s")
    return cat, w


def time_path(tpcf, torch, dev, precision, steps, warmup, autotune=True, fixed=None):
    """Times `steps` hot-path steps; returns (ms_per_step, mean sweep ms, stats, zeta, tuning).
    The autotuner (if on) runs once before the warmup, outside the timed steps; `fixed` =
    (points per cell, waves per CU) sets the tuning instead."""
    ctx = make_ctx(tpcf, torch.cuda.current_stream())
    ctx.set_bins(NB, RMIN, RMAX, LMAX)
    ctx.set_precision(precision)
    if fixed:
        ctx.set_tuning(fixed[0], int(fixed[1]))

    def step():
        ctx.set_catalog(*dev[:3], dev[3], box=BOX, periodic=True)
        return ctx.compute_zeta(device_output=True)

    tuning = {"points_per_cell": fixed[0], "waves_per_cu": int(fixed[1]), "source": "--tuning"} if fixed else None
    if autotune and not fixed:
        ctx.set_catalog(*dev[:3], dev[3], box=BOX, periodic=True)
        t0 = time.perf_counter()
        tuning = ctx.autotune()
        tuning["seconds"] = time.perf_counter() - t0
        log(f"[bench] {precision} autotune: {tuning}")

    for i in range(warmup):
        step()
        log(f"[bench] {precision} warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    sweep_ms = []
    t0 = time.perf_counter()
    for i in range(steps):
        z = step()
        sweep_ms.append(ctx.stats()["ms_sweep"])
        log(f"[bench] {precision} step {i + 1}/{steps} sweep {sweep_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    st = ctx.stats()
    st["bin_pairs"] = ctx.pair_sums()[0][0]
    zc = z.cpu().numpy()
    ctx.close()
    return ms, float(np.mean(sweep_ms)), st, zc, tuning


ORACLE_FIXTURE = os.path.join(ROOT, "tests", "golden", "lognormal1e6_oracle.txt")
TOL = {"mixed": 1e-5, "fp64": 1e-10}


def rel_errors(z, ref):
    """Error per (l, r1, r2) relative to max |ref_l| over the bin pairs of l: the per-l maxima and
    the worst (l, r1, r2)."""
    L1 = ref.shape[0]
    scale = np.abs(ref).reshape(L1, -1).max(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    e = np.abs(z - ref) / scale[:, None, None]
    l, b1, b2 = np.unravel_index(int(np.argmax(e)), e.shape)
    return ([float(v) for v in e.reshape(L1, -1).max(axis=1)],
            {"l": int(l), "r1_bin": int(b1), "r2_bin": int(b2), "rel_err": float(e[l, b1, b2])})


def oracle_check(cat, w, results):
    """Compares full-catalogue results with the stored FP64 oracle zeta of the same catalogue
    (tests/golden/lognormal1e6_oracle.txt, written by the oracle alone). results: precision ->
    (zeta, stats with n_pairs and bin_pairs). None when the fixture is absent."""
    if not os.path.exists(ORACLE_FIXTURE):
        return None
    import importlib.util

    spec = importlib.util.spec_from_file_location(
        "oracle_fixture", os.path.join(ROOT, "tests", "golden", "make_lognormal1e6_oracle.py"))
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    gold = fx.read(ORACLE_FIXTURE)
    out = {"fixture": os.path.relpath(ORACLE_FIXTURE, ROOT),
           "catalogue_sha256_match": fx.catalogue_hash(cat, w) == gold["sha256"],
           "tolerance": TOL, "per_l": {}, "worst": {}}
    if not out["catalogue_sha256_match"]:
        return out
    ok = True
    for prec, (z, st) in results.items():
        per_l, worst = rel_errors(z, gold["zeta"])
        out["per_l"][prec] = per_l
        out["worst"][prec] = worst
        out.setdefault("pairs_match", {})[prec] = int(st["n_pairs"]) == gold["npairs"]
        out.setdefault("bin_pairs_match", {})[prec] = bool(np.array_equal(st["bin_pairs"], gold["bin_pairs"]))
        ok = ok and worst["rel_err"] <= TOL[prec] and out["pairs_match"][prec] and out["bin_pairs_match"][prec]
    out["within_tolerance"] = ok
    return out


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision, profile=TRAFFIC_PROFILE):
    """HBM bytes per sweep launch from the committed counter profile, if it was taken on the
    kernel source as it is now; None otherwise."""
    if not os.path.exists(profile):
        return None
    vals = {}
    for line in open(profile):
        if line.startswith("- `") and "`: " in line:
            k, v = line[3:].split("`: ", 1)
            vals[k] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        fetch = float(vals[f"{precision}_fetch_bytes"])
        write = float(vals[f"{precision}_write_bytes"])
    except (KeyError, ValueError):
        return None
    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "source": os.path.relpath(profile, ROOT)}


def cpu_baseline_parallel(cat, w, seconds):
    """Oracle on a random primary sample, OpenMP over primaries inside the oracle."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(12345)
    # one primary per thread to calibrate the sample size
    sample = np.sort(rng.choice(cat.n, size=threads, replace=False))
    perm = np.concatenate([sample, np.setdiff1d(np.arange(cat.n), sample)])
    x, y, z, ww = cat.x[perm], cat.y[perm], cat.z[perm], w[perm]
    t0 = time.perf_counter()
    r = oracle.zeta(x, y, z, ww, BOX, True, NB, RMIN, RMAX, LMAX, 0, threads, threads=threads)
    t_cal = time.perf_counter() - t0
    per = t_cal / threads  # seconds per primary per thread-equivalent wall
    k = max(threads, int(seconds / max(per, 1e-6)))
    k = min(k, cat.n)
    sample = np.sort(rng.choice(cat.n, size=k, replace=False))
    perm = np.concatenate([sample, np.setdiff1d(np.arange(cat.n), sample)])
    x, y, z, ww = cat.x[perm], cat.y[perm], cat.z[perm], w[perm]
    t0 = time.perf_counter()
    r = oracle.zeta(x, y, z, ww, BOX, True, NB, RMIN, RMAX, LMAX, 0, k, threads=threads)
    el = time.perf_counter() - t0
    return r.npairs, k, el, threads


def cpu_baseline_one_thread(cat, w, nprim=8):
    """The same oracle on one thread: nprim random primaries (seed 54321) against all secondaries."""
    import oracle

    rng = np.random.default_rng(54321)
    sample = np.sort(rng.choice(cat.n, size=nprim, replace=False))
    perm = np.concatenate([sample, np.setdiff1d(np.arange(cat.n), sample)])
    x, y, z, ww = cat.x[perm], cat.y[perm], cat.z[perm], w[perm]
    t0 = time.perf_counter()
    r = oracle.zeta(x, y, z, ww, BOX, True, NB, RMIN, RMAX, LMAX, 0, nprim, threads=1)
    return r.npairs, time.perf_counter() - t0


def _mock(args):
    """One batch mock (runs in a worker process, before the parent touches the GPU)."""
    import catalogs

    i, n = args
    c = catalogs.lognormal(int(n), BOX, int(i), grid=256)
    return c.x, c.y, c.z


def _map_values(args):
    """Values of one batch map (worker process, before the parent touches the GPU)."""
    import catalogs

    seed, nside = args
    x, y, z = catalogs.healpix_centres(nside)
    return catalogs.sphere_field(x, y, z, seed)


def run_sphere_batch(args):
    """Batch of maps: --mocks full-sky HEALPix nside-512 maps (3,145,728 pixels each) with map
    values from seeds 0..M-1, 20 bins [10, 200) arcmin, m_max = 8, mixed, one persistent launch
    per call, captured as a HIP graph on a non-default stream and replayed."""
    import multiprocessing as mp

    import catalogs

    nside, nb, mmax = 512, 20, 8
    arcmin = math.pi / (180.0 * 60.0)
    tmin, tmax = 10 * arcmin, 200 * arcmin
    M = args.mocks
    t0 = time.time()
    x, y, z = catalogs.healpix_centres(nside)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        vals = pool.map(_map_values, [(i, nside) for i in range(M)], chunksize=1)
    n = len(x)
    log(f"[bench] {M} maps of {n} pixels generated in {time.time() - t0:.1f}s on {workers} processes")
    off = np.arange(M + 1, dtype=np.int64) * n

    import torch

    import paper_2604_08855_amd as tpcf

    dev = [torch.from_numpy(np.tile(a, M)).cuda() for a in (x, y, z)] + \
          [torch.from_numpy(np.concatenate(vals)).cuda()]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = make_ctx(tpcf, stream)
        ctx.set_bins(nb, tmin, tmax, mmax)
        ctx.set_precision("mixed")
        ctx.set_sphere_catalog(*[t[:n] for t in dev])
        tuning = None if args.no_autotune else ctx.autotune()
        log(f"[bench] sphere batch autotune on map 0: {tuning}")
        for i in range(args.warmup):
            ctx.compute_sphere_batch(off, *dev, device_output=True)
            stream.synchronize()
        times = []
        for i in range(args.steps):
            t1 = time.perf_counter()
            zb = ctx.compute_sphere_batch(off, *dev, device_output=True)
            stream.synchronize()
            times.append(time.perf_counter() - t1)
            log(f"[bench] sphere batch step {i + 1}/{args.steps}: {times[-1]:.2f}s")
        st = ctx.stats()
        zb = zb.cpu().numpy()
        # the first and last map, each run alone, against their batch slices
        check = {}
        for k in (0, M - 1):
            ctx.set_sphere_catalog(*[t[off[k]:off[k + 1]] for t in dev])
            z1 = ctx.compute_zeta(device_output=True).cpu().numpy()
            check[f"map{k}"] = float(np.abs(z1 - zb[k]).max() / np.abs(z1).max())
        ctx.close()
    ms = float(np.mean(times)) * 1000.0
    pairs = st["n_pairs"]
    f_pair, f_prim = 4 * (2 * mmax + 1), 2 * nb * nb * (2 * mmax + 1)
    achieved = (pairs * f_pair + M * n * f_prim) / (ms / 1000.0) / 1e12
    out = {
        "metric": "primary-secondary pairs/sec (m_max=8, 20 angular bins), mixed, batch of full-sky maps",
        "value": pairs / (ms / 1000.0), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{M} HEALPix nside {nside} maps (seeds 0..{M - 1}), log-normal map values, "
                               "20 bins [10,200) arcmin, m_max=8, mixed, one graph-replayed launch",
                   "maps": M, "n_points": M * n, "pairs_per_step": pairs, "tuning": tuning},
        "batch_slice_vs_single_run_rel_err": check,
        "roofline": {"bound": "alu", "kernel": "sweep_kernel<8,false,true>", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": None},
    }
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Batch form: independent log-normal mocks (seeds 0..M-1, sizes log-uniform in [2e5, 2e6]
    from seed 1000), L = 1000 periodic, unit weights, 20 bins [10, 200), l_max = 10, mixed, one
    persistent launch per call, captured as a HIP graph on a non-default stream and replayed. The
    autotuner runs on one mock, the pair-weighted median one."""
    import multiprocessing as mp

    import catalogs

    sizes = catalogs.mock_sizes(args.mocks, 2e5, 2e6, 1000)
    t0 = time.time()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        cats = pool.map(_mock, list(enumerate(sizes)), chunksize=1)
    log(f"[bench] {len(cats)} mocks, {int(sizes.sum())} points generated in {time.time() - t0:.1f}s "
        f"on {workers} processes")
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    import torch

    import paper_2604_08855_amd as tpcf

    dev = [torch.from_numpy(np.concatenate([c[k] for c in cats])).cuda() for k in range(3)]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = make_ctx(tpcf, stream)
        ctx.set_bins(NB, RMIN, RMAX, LMAX)
        ctx.set_precision("mixed")
        tuning = None
        if not args.no_autotune:
            # tuned on the pair-weighted median mock (pairs grow as n^2, so the larger mocks carry
            # most of the sweep)
            order = np.argsort(sizes)
            cum = np.cumsum(sizes[order].astype(np.float64) ** 2)
            k = int(order[int(np.searchsorted(cum, 0.5 * cum[-1]))])
            ctx.set_catalog(*[t[off[k]:off[k + 1]] for t in dev], None, box=BOX, periodic=True)
            tuning = ctx.autotune()
            log(f"[bench] batch autotune on mock {k} ({sizes[k]} points): {tuning}")
        for i in range(args.warmup):
            ctx.compute_batch(off, *dev, None, BOX, True, device_output=True)
            stream.synchronize()
            log(f"[bench] batch warmup {i + 1}/{args.warmup} done")
        times, sweeps = [], []
        for i in range(args.steps):
            t1 = time.perf_counter()
            zb = ctx.compute_batch(off, *dev, None, BOX, True, device_output=True)
            stream.synchronize()
            times.append(time.perf_counter() - t1)
            sweeps.append(ctx.stats()["ms_sweep"])
            log(f"[bench] batch step {i + 1}/{args.steps}: {times[-1]:.2f}s")
        st = ctx.stats()
        zb = zb.cpu().numpy()
        # the smallest and largest mock, each run alone, against their batch slices
        check = {}
        for k in (int(np.argmin(sizes)), int(np.argmax(sizes))):
            ctx.set_catalog(*[t[off[k]:off[k + 1]] for t in dev], None, box=BOX, periodic=True)
            z1 = ctx.compute_zeta(device_output=True).cpu().numpy()
            check[f"mock{k}_n{int(sizes[k])}"] = float(np.abs(z1 - zb[k]).max() / np.abs(z1).max())
        ctx.close()
    ms = float(np.mean(times)) * 1000.0
    pairs = st["n_pairs"]
    flops = pairs * F_PAIR + int(sizes.sum()) * F_PRIM
    achieved = flops / (ms / 1000.0) / 1e12
    out = {
        "metric": "primary-secondary pairs/sec (l_max=10, 20 bins), mixed, batch form",
        "value": pairs / (ms / 1000.0),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batch: {args.mocks} log-normal mocks (seeds 0..{args.mocks - 1}), sizes "
                        "log-uniform [2e5, 2e6] (seed 1000), L=1000 periodic, w=1, 20 bins [10,200), "
                        "l_max=10, mixed, one persistent launch replayed from a HIP graph",
            "mocks": args.mocks,
            "n_points": int(sizes.sum()),
            "pairs_per_step": pairs,
            "candidates_per_step": st["n_candidates"],
            "tuning": tuning,
        },
        "graph_ms": float(np.mean(sweeps)),
        "batch_vs_single_max_rel_diff": check,
        "roofline": {
            "bound": "alu",
            "kernel": "sweep_kernel<10,false,false>",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "peak_without_packed_fp32": PEAK_FP32_UNPACKED_TFLOPS,
            "frac_without_packed_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
            "traffic": None,
            "flops_per_launch": flops,
        },
    }
    print(json.dumps(out), flush=True)


def run_dmr(args):
    """Large single catalogue: 4e6 log-normal data points (w = 1) plus 1.6e7 uniform randoms
    (w = -N_d/N_r) in a non-periodic cube of side 2000, 20 bins [10, 200), l_max = 10; mixed and
    FP64, with primary ranges of data and of randoms checked against the oracle."""
    import catalogs
    import oracle

    t0 = time.time()
    cat = catalogs.data_minus_randoms(4_000_000, 16_000_000, 2000.0, 0, 1, grid=256)
    log(f"[bench] data-minus-randoms catalogue ({cat.n} points) generated in {time.time() - t0:.1f}s")

    import torch

    import paper_2604_08855_amd as tpcf

    dev = [torch.from_numpy(a).cuda() for a in (cat.x, cat.y, cat.z, cat.w)]
    torch.cuda.synchronize()
    res, zfull = {}, {}
    ranges = [(0, 24), (4_000_000, 4_000_024)]  # 24 data primaries, 24 random primaries
    for prec, steps in (("mixed", args.steps), ("fp64", 1)):
        ctx = make_ctx(tpcf, torch.cuda.current_stream())
        ctx.set_bins(NB, RMIN, RMAX, LMAX)
        ctx.set_precision(prec)
        ctx.set_catalog(*dev, box=cat.box, periodic=False)
        tuning = None if args.no_autotune else ctx.autotune()
        ctx.compute_zeta(device_output=True)  # warmup
        torch.cuda.synchronize()
        times, sweeps = [], []
        for i in range(steps):
            t1 = time.perf_counter()
            ctx.set_catalog(*dev, box=cat.box, periodic=False)
            zN = ctx.compute_zeta(device_output=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            sweeps.append(ctx.stats()["ms_sweep"])
            log(f"[bench] dmr {prec} step {i + 1}/{steps}: {times[-1]:.2f}s")
        st = ctx.stats()
        npairs, _ = ctx.pair_sums()
        zfull[prec] = zN.cpu().numpy()
        extra = {"pair_sums_total_equals_pair_count": int(npairs.sum()) == st["n_pairs"]}
        if prec == "mixed":
            # randoms alone (weight +N_d/N_r) and the edge-corrected multipoles N / R
            nd = 4_000_000
            t1 = time.perf_counter()
            ctx.set_catalog(dev[0][nd:], dev[1][nd:], dev[2][nd:], -dev[3][nd:], box=cat.box, periodic=False)
            zR = ctx.compute_zeta(device_output=True)
            torch.cuda.synchronize()
            extra["randoms_only_s"] = time.perf_counter() - t1
            t1 = time.perf_counter()
            zc = ctx.edge_correct(zN, zR)
            torch.cuda.synchronize()
            extra["edge_correct_ms"] = (time.perf_counter() - t1) * 1000.0
            zrr = ctx.edge_correct(zR, zR).cpu().numpy()
            unit = np.zeros_like(zrr)
            unit[0] = 1.0
            extra["edge_correct_R_over_R_max_abs_dev_from_1"] = float(np.abs(zrr - unit).max())
            zc = zc.cpu().numpy()
            extra["edge_corrected_zeta0_diag_first_bins"] = [float(zc[0, b, b]) for b in range(3)]
            ctx.set_catalog(*dev, box=cat.box, periodic=False)
        errs = []
        for b0, b1 in ranges:
            zg = ctx.compute_zeta_range(b0, b1)
            ref = oracle.zeta(cat.x, cat.y, cat.z, cat.w, cat.box, False, NB, RMIN, RMAX, LMAX, b0, b1).zeta
            scale = np.abs(ref).reshape(LMAX + 1, -1).max(axis=1)
            errs.append(float((np.abs(zg - ref).reshape(LMAX + 1, -1).max(axis=1) / scale).max()))
        ctx.close()
        ms = float(np.mean(times)) * 1000.0
        res[prec] = {"value": st["n_pairs"] / (ms / 1000.0), "ms_per_step": ms, "sweep_ms": float(np.mean(sweeps)),
                     "pairs_per_step": st["n_pairs"], "candidates_per_step": st["n_candidates"],
                     "tuning": tuning, "max_rel_err_vs_oracle_on_sampled_ranges": max(errs), **extra}
        log(f"[bench] dmr {prec}: {res[prec]}")
    m = res["mixed"]
    err_vs_fp64, worst_vs_fp64 = rel_errors(zfull["mixed"], zfull["fp64"])
    log(f"[bench] dmr mixed vs fp64 worst {worst_vs_fp64}")
    flops = m["pairs_per_step"] * F_PAIR + cat.n * F_PRIM
    achieved = flops / (m["sweep_ms"] / 1000.0) / 1e12
    out = {
        "metric": "primary-secondary pairs/sec (l_max=10, 20 bins), mixed, data minus randoms",
        "value": m["value"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "4e6 log-normal data (w=1) + 1.6e7 uniform randoms (w=-0.25), non-periodic "
                               "cube L=2000, 20 bins [10,200), l_max=10, mixed", "n_points": cat.n,
                   "pairs_per_step": m["pairs_per_step"], "candidates_per_step": m["candidates_per_step"],
                   "tuning": m["tuning"]},
        "fp64": res["fp64"],
        "mixed_over_fp64_speedup": m["value"] / res["fp64"]["value"],
        "max_rel_err_vs_oracle_on_sampled_ranges": {k: v["max_rel_err_vs_oracle_on_sampled_ranges"]
                                                    for k, v in res.items()},
        "max_rel_err_mixed_vs_fp64_per_l": err_vs_fp64,
        "worst_mixed_vs_fp64": worst_vs_fp64,
        "roofline": {"bound": "alu", "kernel": "sweep_kernel<10,false,false>", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "peak_without_packed_fp32": PEAK_FP32_UNPACKED_TFLOPS,
                     "frac_without_packed_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                     "traffic": None, "flops_per_launch": flops},
    }
    print(json.dumps(out), flush=True)


def run_pivots(args):
    """Shared pivots (the paper's approximate speed-up) on the main catalogue: the exact mixed and
    FP64 paths, then pivot cells of 0.5, 1 and 2 mean separations (5, 10, 20 Mpc/h), each timed
    over the same steps; the error is max over l of max|zeta_l - exact FP64| / max|exact FP64|."""
    import torch

    import paper_2604_08855_amd as tpcf

    cat, w = make_catalog()
    dev = [torch.from_numpy(a).cuda() for a in (cat.x, cat.y, cat.z, w)]
    torch.cuda.synchronize()

    def timed(prec, side):
        ctx = make_ctx(tpcf, torch.cuda.current_stream())
        ctx.set_bins(NB, RMIN, RMAX, LMAX)
        ctx.set_precision(prec)
        ctx.set_tuning(16.0, 12 if prec == "mixed" else 8)  # the library's default waves per CU
        ctx.set_pivot_cell(side)
        ctx.set_catalog(*dev[:3], dev[3], box=BOX, periodic=True)
        z = ctx.compute_zeta(device_output=True)  # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.set_catalog(*dev[:3], dev[3], box=BOX, periodic=True)
            z = ctx.compute_zeta(device_output=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        st = ctx.stats()
        ctx.close()
        return ms, st, z.cpu().numpy()

    ms_ex, st_ex, z_ex = timed("mixed", 0.0)
    ms64, _, z64 = timed("fp64", 0.0)

    def err(z):
        return float(max(np.abs(z[l] - z64[l]).max() / np.abs(z64[l]).max() for l in range(LMAX + 1)))

    rows = [{"pivot_cell": 0.0, "ms_per_step": ms_ex, "pivots": st_ex["n_primaries"], "pairs": st_ex["n_pairs"],
             "speedup": 1.0, "max_rel_err_vs_exact_fp64": err(z_ex)}]
    log(f"[bench] exact mixed {ms_ex:.1f} ms, FP64 {ms64:.1f} ms")
    sep = BOX / N ** (1.0 / 3.0)
    for f in (0.5, 1.0, 2.0):
        ms, st, z = timed("mixed", f * sep)
        rows.append({"pivot_cell": f * sep, "ms_per_step": ms, "pivots": st["n_primaries"], "pairs": st["n_pairs"],
                     "speedup": ms_ex / ms, "max_rel_err_vs_exact_fp64": err(z)})
        log(f"[bench] pivot cell {f * sep:.1f}: {rows[-1]}")
    best = rows[2]  # one mean separation, the paper's default
    out = {
        "metric": "primary-secondary pairs/sec equivalent (exact-pair count / time), shared pivots at the mean separation",
        "value": st_ex["n_pairs"] / (best["ms_per_step"] / 1000.0), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "lognormal N=1e6 L=1000 periodic, w=1+0.1N(0,1), 20 bins [10,200), l_max=10, mixed, "
                               "shared pivots", "mean_separation": sep},
        "sweep_of_pivot_cells": rows, "exact_fp64_ms_per_step": ms64,
    }
    print(json.dumps(out), flush=True)


def run_sphere_large(args):
    """The sphere workload at a larger map (--nside, e.g. 4096: 201,326,592 pixels), same bins and
    m_max as the nside-1024 form, mixed only: the exact sweep over --chunks primary ranges (their
    zeta add up to the whole; each range reports its progress), shared pivots at the pivot cells of
    --pivot-cells (in mean pixel separations), and sampled primary ranges against the oracle."""
    import catalogs
    import oracle

    nside, nb, mmax = args.nside, 20, 8
    arcmin = math.pi / (180.0 * 60.0)
    tmin, tmax = 10 * arcmin, 200 * arcmin
    t0 = time.time()
    x, y, z = catalogs.healpix_centres(nside)
    n = len(x)
    log(f"[bench] HEALPix nside {nside}: {n} pixel centres in {time.time() - t0:.1f}s")
    field = catalogs.sphere_field_sampler(2604)
    w = np.empty(n)
    step = 1 << 24
    for a in range(0, n, step):
        b = min(n, a + step)
        w[a:b] = field(x[a:b], y[a:b], z[a:b])
        log(f"[bench] map values {b}/{n} ({time.time() - t0:.1f}s)")

    import torch

    import paper_2604_08855_amd as tpcf

    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, w)]
    torch.cuda.synchronize()
    ctx = make_ctx(tpcf, torch.cuda.current_stream())
    ctx.set_bins(nb, tmin, tmax, mmax)
    ctx.set_precision("mixed")
    ppc, wpc = (float(v) for v in (args.tuning or "16,12").split(","))
    ctx.set_tuning(ppc, int(wpc))
    t1 = time.perf_counter()
    ctx.set_sphere_catalog(*dev)
    torch.cuda.synchronize()
    t_stage = time.perf_counter() - t1
    zsum = np.zeros((mmax + 1, nb, nb))
    pairs, cands, t_sweep = 0, 0, 0.0
    C = args.chunks
    K = C if args.exact_chunks <= 0 else min(C, args.exact_chunks)
    # K of the C primary ranges, evenly spaced (ring order: latitude bands across the sky)
    for k in sorted({C * i // K for i in range(K)}):
        a, b = n * k // C, n * (k + 1) // C
        t1 = time.perf_counter()
        zsum += ctx.compute_zeta_range(a, b)
        t_sweep += time.perf_counter() - t1
        st = ctx.stats()
        pairs += st["n_pairs"]
        cands += st["n_candidates"]
        log(f"[bench] exact range {k + 1}/{C}: {st['n_pairs']} pairs, {(time.perf_counter() - t1):.1f}s")
    full = K == C
    # all ranges: staging and sweep; a sample of ranges: the sweep rate over those ranges, and the
    # whole-map time scaled from it
    value = pairs / (t_stage + t_sweep) if full else pairs / t_sweep
    t_exact = t_stage + t_sweep * (C / K)
    log(f"[bench] exact ({K} of {C} ranges): {pairs} pairs in {t_sweep:.1f}s (+{t_stage:.1f}s staging), "
        f"{value:.3e} pairs/s")
    errs = []
    for a in (0, n // 2, n - 8):
        zg = ctx.compute_zeta_range(a, a + 8)
        ref = oracle.zeta_sphere(x, y, z, w, nb, tmin, tmax, mmax, a, a + 8).zeta
        scale = np.abs(ref).reshape(mmax + 1, -1).max(axis=1)
        errs.append(float((np.abs(zg - ref).reshape(mmax + 1, -1).max(axis=1) / scale).max()))
        log(f"[bench] oracle check [{a}, {a + 8}): {errs[-1]:.2e}")
    ctx.close()
    sep = math.sqrt(4.0 * math.pi / n)
    piv = []
    for f in (float(v) for v in args.pivot_cells.split(",") if v):
        ctx = make_ctx(tpcf, torch.cuda.current_stream())
        ctx.set_bins(nb, tmin, tmax, mmax)
        ctx.set_precision("mixed")
        ctx.set_tuning(ppc, int(wpc))
        ctx.set_pivot_cell(f * sep)
        t1 = time.perf_counter()
        ctx.set_sphere_catalog(*dev)
        zp = ctx.compute_zeta()
        el = time.perf_counter() - t1
        st = ctx.stats()
        e = (float(max(np.abs(zp[k] - zsum[k]).max() / np.abs(zsum[k]).max() for k in range(mmax + 1)))
             if full else None)
        piv.append({"pivot_cell": f * sep, "pivots": st["n_primaries"], "seconds": el,
                    "speedup_vs_exact": t_exact / el, "max_rel_err_vs_exact_mixed": e})
        log(f"[bench] shared pivots {piv[-1]}")
        ctx.close()
    out = {
        "metric": f"primary-secondary pairs/sec (m_max=8, 20 angular bins), mixed, full-sky map nside {nside}",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": t_exact * 1000.0, "higher_is_better": True, "scaling": "weak",
        "exact_primary_ranges_run": f"{K} of {C}" + ("" if full else " (value: sweep rate over those ranges; "
                                                      "ms_per_step: staging + sweep scaled to all ranges)"),
        "staging_seconds": t_stage,
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"HEALPix nside {nside} full sky ({n} pixels), log-normal map values, 20 bins "
                               f"[10,200) arcmin, m_max=8, mixed, {C} primary ranges", "n_points": n,
                   "pairs_per_step": pairs, "candidates_per_step": cands,
                   "tuning": {"points_per_cell": ppc, "waves_per_cu": int(wpc)},
                   "phase_aligned": {-1: "auto", 0: "off", 1: "on"}[args.phase_aligned]},
        "max_rel_err_vs_oracle_on_sampled_ranges": max(errs),
        "shared_pivots": piv,
    }
    print(json.dumps(out), flush=True)


def calibration_copy(torch, mib):
    """A plain device copy of `mib` MiB: its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters."""
    if mib <= 0:
        return
    src = torch.ones(mib * 2**20 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {mib} MiB done")


def run_sphere(args):
    """The paper's own geometry: a full-sky HEALPix map, nside 1024 (12,582,912 pixels), map values
    rho - 1 of a log-normal field (sigma_lnrho 0.5) sampled on the sphere, 20 angular bins in
    [10, 200) arcmin, m_max = 8; mixed and FP64; three primary ranges checked against the oracle."""
    import catalogs
    import oracle

    nside, nb, mmax = 1024, 20, 8
    arcmin = math.pi / (180.0 * 60.0)
    tmin, tmax = 10 * arcmin, 200 * arcmin
    t0 = time.time()
    m = catalogs.sphere_map(nside, 2604)
    log(f"[bench] HEALPix nside {nside} map ({m.n} pixels) generated in {time.time() - t0:.1f}s")

    import torch

    import paper_2604_08855_amd as tpcf

    dev = [torch.from_numpy(a).cuda() for a in (m.x, m.y, m.z, m.w)]
    torch.cuda.synchronize()
    calibration_copy(torch, args.copy_calibration_mib)
    res, zfull, tunings = {}, {}, {}
    ranges = [(0, 24), (m.n // 2, m.n // 2 + 24), (m.n - 24, m.n)]
    for prec, steps in (("mixed", args.steps), ("fp64", max(1, min(args.steps, 2)))):
        ctx = make_ctx(tpcf, torch.cuda.current_stream())
        ctx.set_bins(nb, tmin, tmax, mmax)
        ctx.set_precision(prec)
        ctx.set_sphere_catalog(*dev)
        if args.tuning:
            ppc, wpc = (float(v) for v in args.tuning.split(","))
            ctx.set_tuning(ppc, int(wpc))
            tuning = {"points_per_cell": ppc, "waves_per_cu": int(wpc), "source": "--tuning"}
        else:
            tuning = None if args.no_autotune else ctx.autotune()
        log(f"[bench] sphere {prec} tuning {tuning}")
        ctx.compute_zeta(device_output=True)  # warmup
        torch.cuda.synchronize()
        times, sweeps = [], []
        for i in range(steps):
            t1 = time.perf_counter()
            ctx.set_sphere_catalog(*dev)
            zs = ctx.compute_zeta(device_output=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            sweeps.append(ctx.stats()["ms_sweep"])
            log(f"[bench] sphere {prec} step {i + 1}/{steps}: {times[-1] * 1000:.1f} ms")
        zfull[prec] = zs.cpu().numpy()
        tunings[prec] = tuning
        st = ctx.stats()
        npairs, _ = ctx.pair_sums()
        errs = []
        for b0, b1 in ranges:
            zg = ctx.compute_zeta_range(b0, b1)
            ref = oracle.zeta_sphere(m.x, m.y, m.z, m.w, nb, tmin, tmax, mmax, b0, b1).zeta
            scale = np.abs(ref).reshape(mmax + 1, -1).max(axis=1)
            errs.append(float((np.abs(zg - ref).reshape(mmax + 1, -1).max(axis=1) / scale).max()))
        ctx.close()
        ms = float(np.mean(times)) * 1000.0
        res[prec] = {"value": st["n_pairs"] / (ms / 1000.0), "ms_per_step": ms, "sweep_ms": float(np.mean(sweeps)),
                     "pairs_per_step": st["n_pairs"], "candidates_per_step": st["n_candidates"],
                     "cells_per_axis": st["cells_per_axis"], "tuning": tuning,
                     "pair_sums_total_equals_pair_count": int(npairs.sum()) == st["n_pairs"],
                     "max_rel_err_vs_oracle_on_sampled_ranges": max(errs)}
        log(f"[bench] sphere {prec}: {res[prec]}")
    # shared pivots (approximate) at 1, 2 and 4 mean pixel separations, mixed
    sep = math.sqrt(4.0 * math.pi / m.n)
    z64 = zfull["fp64"]
    piv = []
    for f in (1.0, 2.0, 4.0):
        ctx = make_ctx(tpcf, torch.cuda.current_stream())
        ctx.set_bins(nb, tmin, tmax, mmax)
        ctx.set_precision("mixed")
        t = tunings["mixed"] or {}
        ctx.set_tuning(float(t.get("points_per_cell", 0.0)), int(t.get("waves_per_cu", 0)))
        ctx.set_pivot_cell(f * sep)
        ctx.set_sphere_catalog(*dev)
        ctx.compute_zeta(device_output=True)  # warmup
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            ctx.set_sphere_catalog(*dev)
            zp = ctx.compute_zeta(device_output=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1000.0 / args.steps
        st = ctx.stats()
        zp = zp.cpu().numpy()
        e = float(max(np.abs(zp[k] - z64[k]).max() / np.abs(z64[k]).max() for k in range(mmax + 1)))
        piv.append({"pivot_cell": f * sep, "pivots": st["n_primaries"], "ms_per_step": ms,
                    "speedup_vs_exact_mixed": res["mixed"]["ms_per_step"] / ms, "max_rel_err_vs_exact_fp64": e})
        log(f"[bench] sphere shared pivots {piv[-1]}")
        ctx.close()
    # a masked map: the band |dec| < 10 deg and the cap dec > 60 deg removed (about 27% of the sky);
    # N from the masked values, R from the mask; corrected against the full sky's own correction
    dec = np.arcsin(np.clip(m.z, -1.0, 1.0))
    keep = torch.from_numpy((np.abs(dec) > np.radians(10.0)) & (dec < np.radians(60.0))).cuda()
    ctx = make_ctx(tpcf, torch.cuda.current_stream())
    ctx.set_bins(nb, tmin, tmax, mmax)
    ctx.set_precision("mixed")
    t = tunings["mixed"] or {}
    ctx.set_tuning(float(t.get("points_per_cell", 0.0)), int(t.get("waves_per_cu", 0)))
    ctx.set_sphere_catalog(*dev[:3], None)
    R_full = ctx.compute_zeta()
    kept = [d[keep] for d in dev]
    t1 = time.perf_counter()
    ctx.set_sphere_catalog(*kept)
    N_mask = ctx.compute_zeta()
    ctx.set_sphere_catalog(*kept[:3], None)
    R_mask = ctx.compute_zeta()
    c_mask = ctx.edge_correct(N_mask, R_mask)
    t_mask = time.perf_counter() - t1
    c_full = ctx.edge_correct(zfull["mixed"], R_full)
    ctx.close()
    diag = np.arange(nb)
    def rel(a):  # per m, max over the diagonal bin pairs of |a - c_full| / max |c_full|
        return [float(np.abs(a[k][diag, diag] - c_full[k][diag, diag]).max() / np.abs(c_full[k][diag, diag]).max())
                for k in range(mmax + 1)]
    masked = {"sky_fraction": float(keep.float().mean().item()), "seconds": t_mask,
              "corrected_vs_full_sky_rel_diff_per_m": rel(c_mask),
              "uncorrected_N_over_R0_vs_full_sky_rel_diff_per_m": rel(N_mask / R_mask[0])}
    log(f"[bench] masked map edge correction {masked}")
    mx = res["mixed"]
    traffic = measured_traffic("mixed", SPHERE_TRAFFIC_PROFILE)
    f_pair = 4 * (2 * mmax + 1)
    f_prim = 2 * nb * nb * (2 * mmax + 1)
    flops = mx["pairs_per_step"] * f_pair + m.n * f_prim
    achieved = flops / (mx["sweep_ms"] / 1000.0) / 1e12
    out = {
        "metric": "primary-secondary pairs/sec (m_max=8, 20 angular bins), mixed, full-sky map",
        "value": mx["value"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": mx["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "HEALPix nside 1024 full sky (12,582,912 pixels), log-normal map values, "
                               "20 bins [10,200) arcmin, m_max=8, mixed", "n_points": m.n,
                   "pairs_per_step": mx["pairs_per_step"], "candidates_per_step": mx["candidates_per_step"],
                   "cells_per_axis": mx["cells_per_axis"], "tuning": mx["tuning"]},
        "fp64": res["fp64"],
        "mixed_over_fp64_speedup": mx["value"] / res["fp64"]["value"],
        "max_rel_err_vs_oracle_on_sampled_ranges": {k: v["max_rel_err_vs_oracle_on_sampled_ranges"]
                                                    for k, v in res.items()},
        "shared_pivots": piv,
        "masked_map_edge_correction": masked,
        "roofline": {"bound": "alu", "kernel": "sweep_kernel<8,false,true>", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "peak_without_packed_fp32": PEAK_FP32_UNPACKED_TFLOPS,
                     "frac_without_packed_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                     "traffic": traffic["bytes"] if traffic else None, "traffic_detail": traffic,
                     "flops_per_launch": flops, "flops_per_pair": f_pair, "flops_per_primary": f_prim,
                     "sweep_ms": mx["sweep_ms"]},
    }
    if args.cpu_seconds > 0:
        threads = len(os.sched_getaffinity(0))
        t1 = time.perf_counter()
        r = oracle.zeta_sphere(m.x, m.y, m.z, m.w, nb, tmin, tmax, mmax, 0, threads, threads=threads)
        per = (time.perf_counter() - t1) / threads
        k = int(min(m.n, max(threads, args.cpu_seconds / max(per, 1e-6))))
        t1 = time.perf_counter()
        r = oracle.zeta_sphere(m.x, m.y, m.z, m.w, nb, tmin, tmax, mmax, 0, k, threads=threads)
        el = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": r.npairs / el, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "oracle_form": "all-pairs: every pixel tested for every primary (no cell "
                                              "grid), FP64",
                               "sample": f"primaries [0, {k}) of the same map against all pixels (brute force "
                                         f"over all secondaries), FP64, {r.npairs} pairs in {el:.1f}s"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default tuning")
    ap.add_argument("--tuning", default="", help="'PPC,WPC' points per cell and waves per CU "
                                                 "instead of the autotuner (profiling runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--workload", choices=["single", "batch", "dmr", "sphere", "sphere-batch", "pivots"],
                    default="single",
                    help="single: the 1e6-point catalogue (default); batch: the mock batch form; "
                         "dmr: 4e6 data + 1.6e7 randoms, non-periodic; sphere: a full-sky HEALPix "
                         "nside 1024 map with angular bins; sphere-batch: --mocks nside-512 maps in "
                         "one launch; pivots: shared pivots (approximate) on the main catalogue")
    ap.add_argument("--mocks", type=int, default=256, help="batch form: number of mocks")
    ap.add_argument("--nside", type=int, default=1024, help="sphere form: HEALPix resolution of the map")
    ap.add_argument("--chunks", type=int, default=16, help="sphere form above nside 1024: primary ranges")
    ap.add_argument("--pivot-cells", default="2,4", help="sphere form above nside 1024: shared-pivot cells "
                                                         "in mean pixel separations")
    ap.add_argument("--phase-aligned", type=int, default=-1, choices=(-1, 0, 1),
                    help="phase-aligned stencil sweeps (-1 by neighbourhood size, 0 off, 1 on)")
    ap.add_argument("--deterministic", action="store_true",
                    help="bit-reproducible results (tpcf_set_deterministic): fixed tiles, fixed-order reduction")
    ap.add_argument("--exact-chunks", type=int, default=0, help="sphere form above nside 1024: time the exact "
                                                                "sum on this many of the --chunks ranges (0: all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    global PHASE_ALIGNED, DETERMINISTIC
    PHASE_ALIGNED = args.phase_aligned
    DETERMINISTIC = args.deterministic
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "dmr":
        run_dmr(args)
        return
    if args.workload == "sphere":
        if args.nside != 1024:
            run_sphere_large(args)
        else:
            run_sphere(args)
        return
    if args.workload == "pivots":
        run_pivots(args)
        return
    if args.workload == "sphere-batch":
        run_sphere_batch(args)
        return

    import torch

    import paper_2604_08855_amd as tpcf

    cat, w = make_catalog()
    dev = [torch.from_numpy(a).cuda() for a in (cat.x, cat.y, cat.z, w)]
    torch.cuda.synchronize()
    calibration_copy(torch, args.copy_calibration_mib)

    tune = not args.no_autotune
    fixed = tuple(float(v) for v in args.tuning.split(",")) if args.tuning else None
    ms, sweep_ms, st, zmix, tmix = time_path(tpcf, torch, dev, "mixed", args.steps, args.warmup, tune, fixed)
    pairs = st["n_pairs"]
    value = pairs / (ms / 1000.0)
    log(f"[bench] mixed: {ms:.1f} ms/step, sweep {sweep_ms:.1f} ms, {pairs} pairs, {value:.3e} pairs/s")

    f64_steps = args.fp64_steps if args.fp64_steps is not None else max(1, min(args.steps, 3))
    ms64, sweep64, st64, z64, t64 = time_path(tpcf, torch, dev, "fp64", f64_steps, 1, tune, fixed)
    value64 = st64["n_pairs"] / (ms64 / 1000.0)
    log(f"[bench] fp64: {ms64:.1f} ms/step, sweep {sweep64:.1f} ms, {value64:.3e} pairs/s")
    err, worst_vs_fp64 = rel_errors(zmix, z64)
    check = oracle_check(cat, w, {"mixed": (zmix, st), "fp64": (z64, st64)})
    if check is None:
        log("[bench] no stored oracle zeta for this catalogue: oracle comparison skipped")
    elif not check["catalogue_sha256_match"]:
        log("[bench] WARNING: the generated catalogue differs from the stored oracle's: comparison skipped")
    elif not check["within_tolerance"]:
        log(f"[bench] WARNING: outside the oracle bars: {check}")
    else:
        log(f"[bench] vs oracle: mixed worst {check['worst']['mixed']}, fp64 worst {check['worst']['fp64']}")

    flops = pairs * F_PAIR + st["n_primaries"] * F_PRIM
    achieved = flops / (sweep_ms / 1000.0) / 1e12
    traffic = measured_traffic("mixed")
    out = {
        "metric": "primary-secondary pairs/sec (l_max=10, 20 bins), mixed vs FP64 GPU at 1e-5 rel err",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "lognormal N=1e6 L=1000 periodic, w=1+0.1N(0,1), 20 bins [10,200), l_max=10, mixed",
            "n_points": N,
            "pairs_per_step": pairs,
            "candidates_per_step": st["n_candidates"],
            "cells_per_axis": st["cells_per_axis"],
            "points_per_cell": N / st["cells_per_axis"] ** 3,
            "waves": st["waves"],
            "tuning": tmix,
            "deterministic": DETERMINISTIC,
        },
        "fp64": {"value": value64, "unit": "pairs/s", "ms_per_step": ms64, "sweep_ms": sweep64,
                 "tuning": t64},
        "mixed_over_fp64_speedup": value / value64,
        "max_rel_err_vs_oracle_per_l": check["per_l"].get("mixed") if check else None,
        "worst_vs_oracle": check["worst"].get("mixed") if check else None,
        "oracle_check": check,
        "max_rel_err_mixed_vs_fp64_per_l": err,
        "worst_mixed_vs_fp64": worst_vs_fp64,
        "grid_ms": st["ms_grid"],
        "roofline": {
            "bound": "alu",
            "kernel": "sweep_kernel<10,false,false>",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "peak_without_packed_fp32": PEAK_FP32_UNPACKED_TFLOPS,
            "frac_without_packed_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_detail": traffic,
            "flops_per_launch": flops,
            "sweep_ms": sweep_ms,
        },
    }
    if args.cpu_seconds > 0:
        cp, nprim, el, threads = cpu_baseline_parallel(cat, w, args.cpu_seconds)
        out["cpu_baseline"] = {
            "value": cp / el,
            "unit": "pairs/s",
            "cores": threads,
            "kind": "oracle",
            "oracle_form": "all-pairs: every secondary tested for every primary (no cell grid), "
                           "trigonometric Y_lm, FP64",
            "sample": f"{nprim} random primaries (seed 12345) of the same 1e6-point catalogue against "
                      f"all 1e6 secondaries (all-pairs oracle), FP64, {cp} pairs in {el:.1f}s",
        }
        log(f"[bench] cpu oracle: {cp / el:.3e} pairs/s on {threads} threads")
        c1, el1 = cpu_baseline_one_thread(cat, w)
        out["cpu_baseline"]["value_one_thread"] = c1 / el1
        out["cpu_baseline"]["sample_one_thread"] = (f"8 random primaries (seed 54321), one thread, {c1} pairs "
                                                    f"in {el1:.1f}s")
        log(f"[bench] cpu oracle, one thread: {c1 / el1:.3e} pairs/s")
    print(json.dumps(out), flush=True)
    if check is not None and check["catalogue_sha256_match"] and not check["within_tolerance"]:
        sys.exit(3)  # the line is printed for the record, but the step did not meet the error bars


if __name__ == "__main__":
    main()
