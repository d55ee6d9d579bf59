"""Writes ``lognormal1e6_oracle.txt``: the FP64 oracle's zeta_l(r1, r2) over the WHOLE
1,000,000-point log-normal catalogue with weights 1 + 0.1 N(0,1) (periodic cube of side
1000 Mpc/h, 20 linear bins over [10, 200), l_max = 10): the estimator of the paper's
Implementation section (per pivot, every neighbour in range fills the multipole bins; the
multipoles are contracted and summed over pivots), summed over every primary.

This script calls only ``catalogs`` (the seeded input generator) and ``oracle``; nothing from
the GPU library. The oracle runs over consecutive primary ranges of ``--chunk`` primaries; each
range's partial zeta, pair counts per bin and pair total are saved under ``--parts`` so an
interrupted run resumes where it stopped, and the partials are added in range order at the end.

The output file holds: the sha256 of the generated x, y, z, w (float64 bytes, in that order),
the in-range ordered pair total, the ordered pair count per bin, and zeta[l][b1][b2] with 17
significant digits. The GPU test regenerates the catalogue, checks the hash and compares the
library's full-catalogue zeta with these values element by element.

Usage: python tests/golden/make_lognormal1e6_oracle.py --parts DIR [--threads T] [--chunk C]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lognormal1e6_oracle.txt")
N, BOX, NB, RMIN, RMAX, LMAX = 1_000_000, 1000.0, 20, 10.0, 200.0, 10


def catalogue():
    """The catalogue, generated exactly as the benchmark generates it."""
    import catalogs

    cat = catalogs.lognormal(N, BOX, 0, grid=256)
    w = catalogs.gaussian_weights(N, 10**6, 1.0, 0.1)
    return cat, w


def catalogue_hash(cat, w) -> str:
    h = hashlib.sha256()
    for a in (cat.x, cat.y, cat.z, w):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def read(path: str = OUT) -> dict:
    """Parses the output file: {'sha256', 'npairs', 'bin_pairs' [NB], 'zeta' [L+1][NB][NB]}."""
    meta, rows = {}, []
    for line in open(path):
        line = line.strip()
        if not line:
            continue
        if line.startswith("#"):
            if ":" in line:
                k, v = line[1:].split(":", 1)
                meta[k.strip()] = v.strip()
            continue
        rows.append([float(t) for t in line.split()])
    z = np.zeros((LMAX + 1, NB, NB))
    for r in rows:
        l, b1 = int(r[0]), int(r[1])
        z[l, b1, :] = r[2:]
    return {"sha256": meta["sha256"], "npairs": int(meta["npairs"]),
            "bin_pairs": np.array([int(t) for t in meta["bin_pairs"].split()], dtype=np.int64),
            "zeta": z}


def main():
    import oracle

    ap = argparse.ArgumentParser()
    ap.add_argument("--parts", required=True, help="directory for the per-range partial results")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=10_000)
    args = ap.parse_args()
    os.makedirs(args.parts, exist_ok=True)

    cat, w = catalogue()
    digest = catalogue_hash(cat, w)
    print(f"catalogue sha256 {digest}", flush=True)
    nchunk = (N + args.chunk - 1) // args.chunk
    zsum = np.zeros((LMAX + 1, NB, NB))
    bins = np.zeros(NB, dtype=np.int64)
    total = 0
    t_start = time.time()
    for c in range(nchunk):
        lo, hi = c * args.chunk, min(N, (c + 1) * args.chunk)
        part = os.path.join(args.parts, f"part_{digest[:12]}_{lo:07d}_{hi:07d}.npz")
        if not os.path.exists(part):
            t0 = time.time()
            r = oracle.zeta(cat.x, cat.y, cat.z, w, BOX, True, NB, RMIN, RMAX, LMAX, lo, hi,
                            want_counts=True, threads=args.threads)
            tmp = part + ".tmp.npz"
            np.savez(tmp, zeta=r.zeta, bins=r.counts.sum(axis=0), npairs=np.int64(r.npairs))
            os.replace(tmp, part)
            el = time.time() - t0
            print(f"range [{lo}, {hi}): {r.npairs} pairs in {el:.1f} s "
                  f"({r.npairs / el:.3e} pairs/s); {c + 1}/{nchunk} done, "
                  f"{time.time() - t_start:.0f} s so far", flush=True)
        d = np.load(part)
        zsum += d["zeta"]
        bins += d["bins"]
        total += int(d["npairs"])
    assert int(bins.sum()) == total

    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle.zeta) over the whole catalogue; written by\n")
        f.write("# tests/golden/make_lognormal1e6_oracle.py (calls only catalogs and oracle).\n")
        f.write("# catalogue: catalogs.lognormal(1000000, 1000.0, seed 0, grid 256), periodic;\n")
        f.write("#   weights catalogs.gaussian_weights(1000000, seed 1000000, 1.0, 0.1)\n")
        f.write("# bins: 20 linear over [10, 200); l_max: 10\n")
        f.write(f"# primaries summed in ranges of {args.chunk}, range partials added in order\n")
        f.write(f"# sha256: {digest}\n")
        f.write(f"# npairs: {total}\n")
        f.write("# bin_pairs: " + " ".join(str(int(v)) for v in bins) + "\n")
        f.write("# rows: l b1 zeta[l][b1][0..19]\n")
        for l in range(LMAX + 1):
            for b1 in range(NB):
                f.write(f"{l} {b1} " + " ".join(f"{v:.17g}" for v in zsum[l, b1]) + "\n")
    print(f"wrote {OUT}: {total} pairs", flush=True)


if __name__ == "__main__":
    main()
