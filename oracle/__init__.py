"""FP64 CPU oracle for the 3PCF multipoles -- test infrastructure.

Only the tests, the smoke check and the benchmark's ``cpu_baseline`` leg may import this
package. The GPU library never calls it and shares no code with it. The C source
(``tpcf_oracle.c``) states the definition it computes and every reading taken where the paper
is silent; this module only loads it with ctypes and converts arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpcf_oracle.c")
_LIB = os.path.join(_HERE, "libtpcf_oracle.so")
# A prebuilt copy of this oracle (for example a sanitizer build made by the tests) replaces the
# default library when TPCF_ORACLE_LIB names it; it is then loaded as it is, never rebuilt.
_LIB_OVERRIDE = os.environ.get("TPCF_ORACLE_LIB", "")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP). Returns the library path."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        i = ctypes.c_int
        lib.oracle_lattice_bits.argtypes = [d, d, i]
        lib.oracle_lattice_bits.restype = i
        lib.oracle_thresholds.argtypes = [i, d, d, d, i, p]
        lib.oracle_thresholds.restype = None
        lib.oracle_snap.argtypes = [i64, p, d, i, i, p]
        lib.oracle_snap.restype = None
        lib.oracle_ylm.argtypes = [i, i64, p, p, p, p, p]
        lib.oracle_ylm.restype = i
        lib.oracle_zeta.argtypes = [i64, p, p, p, p, d, i, i, d, d, i, i64, i64, p, p, p, p, i]
        lib.oracle_zeta.restype = i
        lib.oracle_pair_sums.argtypes = [i64, p, p, p, p, d, i, i, d, d, i64, i64, p, p, i]
        lib.oracle_pair_sums.restype = i
        lib.oracle_edge_correct.argtypes = [i, i, i, p, p, p]
        lib.oracle_edge_correct.restype = i
        lib.oracle_zeta_sphere.argtypes = [i64, p, p, p, p, i, d, d, i, i64, i64, p, p, p, i]
        lib.oracle_zeta_sphere.restype = i
        lib.oracle_zeta_pivots.argtypes = [i64, p, p, p, p, d, i, i, d, d, i, d, p, p, p, p, p, i]
        lib.oracle_zeta_pivots.restype = i
        lib.oracle_zeta_sphere_pivots.argtypes = [i64, p, p, p, p, i, d, d, i, d, p, p, p, i]
        lib.oracle_degenerate.argtypes = [i64, p, p, p, p, d, i, i, d, d, i, i64, i64, p, i]
        lib.oracle_degenerate.restype = i
        lib.oracle_degenerate_sphere.argtypes = [i64, p, p, p, p, i, d, d, i, i64, i64, p, i]
        lib.oracle_degenerate_sphere.restype = i
        lib.oracle_zeta_sphere_pivots.restype = i
        lib.oracle_edge_correct_sphere.argtypes = [i, i, i, p, p, p]
        lib.oracle_edge_correct_sphere.restype = i
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice_bits(box: float, rmax: float, periodic: bool) -> int:
    return int(_load().oracle_lattice_bits(float(box), float(rmax), int(bool(periodic))))


def thresholds(nbins: int, rmin: float, rmax: float, box: float, K: int) -> np.ndarray:
    T = np.zeros(nbins + 1, dtype=np.uint64)
    _load().oracle_thresholds(int(nbins), float(rmin), float(rmax), float(box), int(K), _ptr(T))
    return T


def snap(x, box: float, K: int, periodic: bool) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.zeros(x.shape[0], dtype=np.int64)
    _load().oracle_snap(x.shape[0], _ptr(x), float(box), int(K), int(bool(periodic)), _ptr(q))
    return q


def ylm(ux, uy, uz, lmax: int) -> np.ndarray:
    """Y_lm of unit vectors; returns complex [n, (lmax+1)^2], column l*l + l + m."""
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    uz = np.ascontiguousarray(uz, dtype=np.float64)
    n = ux.shape[0]
    nc = (lmax + 1) ** 2
    re = np.zeros((n, nc))
    im = np.zeros((n, nc))
    rc = _load().oracle_ylm(int(lmax), n, _ptr(ux), _ptr(uy), _ptr(uz), _ptr(re), _ptr(im))
    if rc:
        raise ValueError("oracle_ylm: invalid lmax")
    return re + 1j * im


class Result:
    def __init__(self, zeta, counts, alm, npairs):
        self.zeta = zeta
        self.counts = counts
        self.alm = alm
        self.npairs = npairs


def zeta(x, y, z, w, box: float, periodic: bool, nbins: int, rmin: float, rmax: float,
         lmax: int, p_begin: int = 0, p_end: int | None = None, want_counts: bool = False,
         want_alm: bool = False, threads: int = 0) -> Result:
    """zeta_l(b1, b2) in FP64 for primaries [p_begin, p_end) against all secondaries."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if p_end is None:
        p_end = n
    npr = p_end - p_begin
    zt = np.zeros((lmax + 1, nbins, nbins))
    counts = np.zeros((npr, nbins), dtype=np.int64) if want_counts else None
    alm = np.zeros((npr, nbins, (lmax + 1) ** 2, 2)) if want_alm else None
    npairs = ctypes.c_int64(0)
    rc = _load().oracle_zeta(
        n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), float(box), int(bool(periodic)), int(nbins),
        float(rmin), float(rmax), int(lmax), int(p_begin), int(p_end), _ptr(zt),
        _ptr(counts) if counts is not None else None,
        _ptr(alm) if alm is not None else None, ctypes.byref(npairs), int(threads))
    if rc:
        raise ValueError("oracle_zeta: invalid arguments")
    a = None if alm is None else alm[..., 0] + 1j * alm[..., 1]
    return Result(zt, counts, a, int(npairs.value))


def pair_sums(x, y, z, w, box: float, periodic: bool, nbins: int, rmin: float, rmax: float,
              p_begin: int = 0, p_end: int | None = None, threads: int = 0):
    """(npairs[nbins] int64, dd[nbins] FP64): ordered pairs per bin and sum of w_p w_j per bin,
    for primaries [p_begin, p_end) against all secondaries (oracle_pair_sums)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if p_end is None:
        p_end = n
    npairs = np.zeros(nbins, dtype=np.int64)
    dd = np.zeros(nbins)
    rc = _load().oracle_pair_sums(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), float(box), int(bool(periodic)),
                                  int(nbins), float(rmin), float(rmax), int(p_begin), int(p_end),
                                  _ptr(npairs), _ptr(dd), int(threads))
    if rc:
        raise ValueError("oracle_pair_sums: invalid arguments")
    return npairs, dd


def edge_correct(N, R):
    """Edge-corrected multipoles zeta solving M(R) zeta = N / R_0 per bin pair
    (oracle_edge_correct); N, R: [(lmax+1), nbins, nbins] or [ncat, (lmax+1), nbins, nbins]."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    if N.shape != R.shape:
        raise ValueError("N and R must have the same shape")
    single = N.ndim == 3
    N4, R4 = (N[None], R[None]) if single else (N, R)
    ncat, L1, nb, _ = N4.shape
    out = np.zeros_like(N4)
    if _load().oracle_edge_correct(ncat, L1 - 1, nb, _ptr(N4), _ptr(R4), _ptr(out)):
        raise ValueError("oracle_edge_correct: invalid arguments")
    return out[0] if single else out


def zeta_sphere(x, y, z, w, nbins: int, theta_min: float, theta_max: float, mmax: int,
                p_begin: int = 0, p_end: int | None = None, want_counts: bool = False,
                threads: int = 0) -> Result:
    """zeta_m(b1, b2), m = 0..mmax, of a projected field on the unit sphere (unit vectors x, y, z;
    angles in radians), primaries [p_begin, p_end) against all points (oracle_zeta_sphere)."""
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if p_end is None:
        p_end = n
    zt = np.zeros((mmax + 1, nbins, nbins))
    counts = np.zeros((p_end - p_begin, nbins), dtype=np.int64) if want_counts else None
    npairs = ctypes.c_int64(0)
    rc = _load().oracle_zeta_sphere(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), int(nbins), float(theta_min),
                                    float(theta_max), int(mmax), int(p_begin), int(p_end), _ptr(zt),
                                    _ptr(counts) if counts is not None else None, ctypes.byref(npairs),
                                    int(threads))
    if rc:
        raise ValueError("oracle_zeta_sphere: invalid arguments")
    return Result(zt, counts, None, int(npairs.value))


def degenerate(x, y, z, w, box: float, periodic: bool, nbins: int, rmin: float, rmax: float, lmax: int,
               p_begin: int = 0, p_end: int | None = None, threads: int = 0) -> np.ndarray:
    """D_l(b) = (2l+1)/(4 pi) sum_p w_p sum_{j in b(p)} w_j^2, the j = k part of zeta_l(b, b)
    (oracle_degenerate); [(lmax+1), nbins]."""
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if p_end is None:
        p_end = n
    D = np.zeros((lmax + 1, nbins))
    rc = _load().oracle_degenerate(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), float(box), int(bool(periodic)),
                                   int(nbins), float(rmin), float(rmax), int(lmax), int(p_begin), int(p_end),
                                   _ptr(D), int(threads))
    if rc:
        raise ValueError("oracle_degenerate: invalid arguments")
    return D


def degenerate_sphere(x, y, z, w, nbins: int, theta_min: float, theta_max: float, mmax: int,
                      p_begin: int = 0, p_end: int | None = None, threads: int = 0) -> np.ndarray:
    """D_m(b) = sum_p w_p sum_{j in b(p)} w_j^2 for every m, the j = k part of zeta_m(b, b) on the
    sphere (oracle_degenerate_sphere); [(mmax+1), nbins]."""
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if p_end is None:
        p_end = n
    D = np.zeros((mmax + 1, nbins))
    rc = _load().oracle_degenerate_sphere(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), int(nbins), float(theta_min),
                                          float(theta_max), int(mmax), int(p_begin), int(p_end), _ptr(D),
                                          int(threads))
    if rc:
        raise ValueError("oracle_degenerate_sphere: invalid arguments")
    return D


class PivotResult:
    """Result of zeta_pivots: zeta, number of pivot groups, pairs, and the group pivots (lattice
    positions [G, 3] and weights [G])."""

    def __init__(self, zeta, ngroups, npairs, gq, gw):
        self.zeta, self.ngroups, self.npairs, self.gq, self.gw = zeta, ngroups, npairs, gq, gw


def zeta_pivots(x, y, z, w, box: float, periodic: bool, nbins: int, rmin: float, rmax: float,
                lmax: int, h: float, threads: int = 0) -> PivotResult:
    """Approximate zeta with pivots shared over cubic pivot cells of side h (oracle_zeta_pivots)."""
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    zt = np.zeros((lmax + 1, nbins, nbins))
    gq = np.zeros((3, max(n, 1)), dtype=np.int64)
    gw = np.zeros(max(n, 1))
    ng, npairs = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = _load().oracle_zeta_pivots(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), float(box), int(bool(periodic)),
                                    int(nbins), float(rmin), float(rmax), int(lmax), float(h), _ptr(zt),
                                    ctypes.byref(ng), ctypes.byref(npairs), _ptr(gq), _ptr(gw), int(threads))
    if rc:
        raise ValueError("oracle_zeta_pivots: invalid arguments")
    G = int(ng.value)
    return PivotResult(zt, G, int(npairs.value), gq[:, :G].T.copy(), gw[:G].copy())


def zeta_sphere_pivots(x, y, z, w, nbins: int, theta_min: float, theta_max: float, mmax: int, h: float,
                       threads: int = 0) -> PivotResult:
    """Approximate zeta_m on the sphere with pivots shared over cubic pivot cells of side h (in the
    units of the unit-vector cube) (oracle_zeta_sphere_pivots)."""
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    n = x.shape[0]
    w = np.ones(n) if w is None else np.ascontiguousarray(w, dtype=np.float64)
    zt = np.zeros((mmax + 1, nbins, nbins))
    ng, npairs = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = _load().oracle_zeta_sphere_pivots(n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), int(nbins), float(theta_min),
                                           float(theta_max), int(mmax), float(h), _ptr(zt), ctypes.byref(ng),
                                           ctypes.byref(npairs), int(threads))
    if rc:
        raise ValueError("oracle_zeta_sphere_pivots: invalid arguments")
    return PivotResult(zt, int(ng.value), int(npairs.value), None, None)


def edge_correct_sphere(N, R):
    """Edge-corrected cosine multipoles c_m of N(phi) / R(phi) on the sphere (oracle_edge_correct_sphere).
    N, R: [(mmax+1), nb, nb] or [ncat, (mmax+1), nb, nb]."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    squeeze = N.ndim == 3
    if squeeze:
        N, R = N[None], R[None]
    out = np.zeros_like(N)
    rc = _load().oracle_edge_correct_sphere(N.shape[0], N.shape[1] - 1, N.shape[2], _ptr(N), _ptr(R), _ptr(out))
    if rc:
        raise ValueError("oracle_edge_correct_sphere: invalid arguments")
    return out[0] if squeeze else out


def zeta_catalog(cat, nbins, rmin, rmax, lmax, **kw) -> Result:
    return zeta(cat.x, cat.y, cat.z, cat.w, cat.box, cat.periodic, nbins, rmin, rmax, lmax, **kw)
