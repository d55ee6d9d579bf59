"""Independent numpy routes used to pin the oracle (test helpers, no shared code with it).

* ``lattice``/``pair_table``: the lattice snapping and integer binning, re-implemented in
  numpy from their stated definition.
* ``zeta_triangles``: the Legendre (triangle) form of the estimator,
      zeta_l(b1,b2) = (2l+1)/(4 pi) sum_p w_p sum_{j in b1} sum_{k in b2} w_j w_k P_l(u_pj . u_pk),
  which follows from the spherical-harmonic addition theorem and needs no Y_lm at all.
* ``pair_counts``: unit-weight per-primary per-bin pair counts.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre


def lattice_bits(box, rmax, periodic):
    m, e = math.frexp(box / rmax)
    K = 25 + (e - 1)
    return max(1, min(K, 32 if periodic else 31))


def snap(x, box, K, periodic):
    sc = math.ldexp(1.0, K) / box
    t = np.floor(np.asarray(x, dtype=np.float64) * sc).astype(np.int64)
    M = 1 << K
    if periodic:
        return np.mod(t, M)
    return np.clip(t, 0, M - 1)


def thresholds(nbins, rmin, rmax, box, K):
    sc = math.ldexp(1.0, K) / box
    delta = (rmax - rmin) / nbins
    T = []
    for k in range(nbins + 1):
        e = rmax if k == nbins else rmin + k * delta
        v = e * sc
        T.append(int(math.ceil(v * v)))
    return np.array(T, dtype=object)


def pair_table(x, y, z, box, periodic, nbins, rmin, rmax, primaries=None):
    """Lists of (p, j, bin, unit vector) for every in-range pair, by the stated definition."""
    n = len(x)
    K = lattice_bits(box, rmax, periodic)
    M = 1 << K
    q = np.stack([snap(x, box, K, periodic), snap(y, box, K, periodic), snap(z, box, K, periodic)], 1)
    T = thresholds(nbins, rmin, rmax, box, K)
    Tlo, Thi = int(T[0]), int(T[-1])
    out = []
    for p in (range(n) if primaries is None else primaries):
        d = q - q[p]
        if periodic:
            d = np.where(d >= M // 2, d - M, d)
            d = np.where(d < -(M // 2), d + M, d)
        for j in range(n):
            if j == p:
                continue
            dx, dy, dz = (int(v) for v in d[j])
            R2 = dx * dx + dy * dy + dz * dz  # Python ints: exact
            if R2 == 0 or R2 < Tlo or R2 >= Thi:
                continue
            b = max(k for k in range(nbins) if int(T[k]) <= R2)
            r = math.sqrt(R2)
            out.append((p, j, b, (dx / r, dy / r, dz / r)))
    return out


def zeta_triangles(x, y, z, w, box, periodic, nbins, rmin, rmax, lmax, primaries=None, drop_jk=False):
    """Legendre form (2l+1)/(4 pi) sum_p w_p sum_{j,k} w_j w_k P_l(u_j . u_k) from the pair table;
    drop_jk leaves out the terms with j = k (one secondary on both legs)."""
    n = len(x)
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    pairs = pair_table(x, y, z, box, periodic, nbins, rmin, rmax, primaries)
    zeta = np.zeros((lmax + 1, nbins, nbins))
    by_p = {}
    for p, j, b, u in pairs:
        by_p.setdefault(p, []).append((j, b, u))
    for p, lst in by_p.items():
        js = np.array([t[0] for t in lst])
        bs = np.array([t[1] for t in lst])
        U = np.array([t[2] for t in lst])
        cosg = np.clip(U @ U.T, -1.0, 1.0)
        ww = np.outer(w[js], w[js])
        if drop_jk:
            np.fill_diagonal(ww, 0.0)
        for l in range(lmax + 1):
            Pl = eval_legendre(l, cosg) * ww
            # accumulate sum over (j,k) into (b_j, b_k)
            acc = np.zeros((nbins, nbins))
            np.add.at(acc, (bs[:, None].repeat(len(js), 1), bs[None, :].repeat(len(js), 0)), Pl)
            zeta[l] += w[p] * (2 * l + 1) / (4 * math.pi) * acc
    return zeta


def pair_counts(x, y, z, box, periodic, nbins, rmin, rmax, primaries=None):
    n = len(x)
    prim = list(range(n)) if primaries is None else list(primaries)
    idx = {p: i for i, p in enumerate(prim)}
    counts = np.zeros((len(prim), nbins), dtype=np.int64)
    for p, j, b, u in pair_table(x, y, z, box, periodic, nbins, rmin, rmax, prim):
        counts[idx[p], b] += 1
    return counts


def pair_sums(x, y, z, w, box, periodic, nbins, rmin, rmax):
    """Ordered pairs and sum of w_p w_j per bin, from the pair table (independent route)."""
    npairs = np.zeros(nbins, dtype=np.int64)
    dd = np.zeros(nbins)
    for p, j, b, u in pair_table(x, y, z, box, periodic, nbins, rmin, rmax):
        npairs[b] += 1
        dd[b] += w[p] * w[j]
    return npairs, dd


# ---------------------------------------------------------------- projected fields on the sphere

def sphere_lattice(x, y, z, nbins, theta_min, theta_max):
    """(q [n, 3], scale, T) of unit vectors on the sphere's lattice, from the stated definition."""
    X = np.stack([np.asarray(a, dtype=np.float64) for a in (x, y, z)], 1) + 2.0
    cmax = 2.0 * math.sin(0.5 * theta_max)
    K = lattice_bits(4.0, cmax, False)
    q = np.stack([snap(X[:, a], 4.0, K, False) for a in range(3)], 1)
    sc = math.ldexp(1.0, K) / 4.0
    dth = (theta_max - theta_min) / nbins
    T = []
    for k in range(nbins + 1):
        th = theta_max if k == nbins else theta_min + k * dth
        v = 2.0 * math.sin(0.5 * th) * sc
        T.append(int(math.ceil(v * v)))
    return q, sc, T


def sphere_triangles_at(qp, wp, skip, q, w, sc, T, nbins, mmax, zeta, counts, sums, row, drop_jk=False):
    """Adds one pivot (lattice point qp, weight wp; point `skip` excluded) to zeta in the basis-free
    triangle form; fills counts[row] and sums[row]."""
    from scipy.special import eval_chebyt
    npv = np.asarray(qp, dtype=np.float64) / sc - 2.0
    npv = npv / np.linalg.norm(npv)
    js, bs, P = [], [], []
    for j in range(len(q)):
        if j == skip:
            continue
        d = [int(a) - int(b) for a, b in zip(q[j], qp)]
        R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
        if R2 == 0 or R2 < T[0] or R2 >= T[-1]:
            continue
        b = max(k for k in range(nbins) if T[k] <= R2)
        dv = np.array(d, dtype=np.float64)
        perp = dv - (dv @ npv) * npv
        js.append(j)
        bs.append(b)
        P.append(perp / np.linalg.norm(perp))
        if counts is not None:
            counts[row, b] += 1
            sums[row, b] += w[j]
    if not js:
        return
    js, bs, P = np.array(js), np.array(bs), np.array(P)
    cosd = np.clip(P @ P.T, -1.0, 1.0)
    ww = np.outer(w[js], w[js])
    if drop_jk:
        np.fill_diagonal(ww, 0.0)
    for m in range(mmax + 1):
        acc = np.zeros((nbins, nbins))
        np.add.at(acc, (bs[:, None].repeat(len(js), 1), bs[None, :].repeat(len(js), 0)),
                  eval_chebyt(m, cosd) * ww)
        zeta[m] += wp * acc


def zeta_sphere_triangles(x, y, z, w, nbins, theta_min, theta_max, mmax, primaries=None, drop_jk=False):
    """zeta_m on the sphere in the basis-free triangle form

        zeta_m(b1, b2) = sum_p w_p sum_{j in b1} sum_{k in b2} w_j w_k cos(m (phi_j - phi_k)),

    where phi_j - phi_k is the angle between the projections of d_j and d_k on the tangent
    plane at the primary, so no tangent basis is needed; cos(m x) = T_m(cos x). Also returns
    the per-primary counts and sums S_p(b) = sum_{j in b} w_j."""
    q, sc, T = sphere_lattice(x, y, z, nbins, theta_min, theta_max)
    n = len(q)
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    zeta = np.zeros((mmax + 1, nbins, nbins))
    counts = np.zeros((n, nbins), dtype=np.int64)
    sums = np.zeros((n, nbins))
    for p in (range(n) if primaries is None else primaries):
        sphere_triangles_at(q[p], w[p], p, q, w, sc, T, nbins, mmax, zeta, counts, sums, p, drop_jk)
    return zeta, counts, sums


# ---------------------------------------------------------------- shared pivots

def pivot_groups(x, y, z, w, box, periodic, rmax, h):
    """Group pivots of the shared-pivot approximation, from its stated definition: groups by
    integer division of the lattice coordinates by Hq = max(1, floor(h 2^K / L)), ordered by
    (gz, gy, gx); pivot at the round-half-up mean lattice position, weight the members' sum."""
    K = lattice_bits(box, rmax, periodic)
    q = np.stack([snap(a, box, K, periodic) for a in (x, y, z)], 1)
    Hq = max(1, int(math.floor(h * (math.ldexp(1.0, K) / box))))
    g = q // Hq
    keys, inv = np.unique(g[:, ::-1], axis=0, return_inverse=True)
    inv = inv.ravel()
    G = len(keys)
    cnt = np.bincount(inv, minlength=G).astype(np.int64)
    sums = np.zeros((G, 3), dtype=np.int64)
    np.add.at(sums, inv, q)
    W = np.zeros(G)
    np.add.at(W, inv, np.asarray(w, dtype=np.float64))
    X = (2 * sums + cnt[:, None]) // (2 * cnt[:, None])
    return X, W, q, K


def zeta_triangles_lattice(qp, wp, qs, ws, K, periodic, T, nbins, lmax):
    """Legendre form of zeta with explicit pivots (lattice points qp, weights wp) and secondaries
    (qs, ws), binning by the integer thresholds T, pairs at zero separation skipped."""
    M = 1 << K
    zeta = np.zeros((lmax + 1, nbins, nbins))
    Tlo, Thi = int(T[0]), int(T[-1])
    for p in range(len(qp)):
        d = qs - qp[p]
        if periodic:
            d = np.where(d >= M // 2, d - M, d)
            d = np.where(d < -(M // 2), d + M, d)
        R2 = (d.astype(object) ** 2).sum(axis=1)
        sel = [j for j in range(len(qs)) if R2[j] != 0 and Tlo <= R2[j] < Thi]
        if not sel:
            continue
        bs = np.array([max(k for k in range(nbins) if int(T[k]) <= R2[j]) for j in sel])
        U = d[sel].astype(np.float64)
        U /= np.linalg.norm(U, axis=1)[:, None]
        cosg = np.clip(U @ U.T, -1.0, 1.0)
        ww = np.outer(ws[sel], ws[sel])
        for l in range(lmax + 1):
            acc = np.zeros((nbins, nbins))
            np.add.at(acc, (bs[:, None].repeat(len(sel), 1), bs[None, :].repeat(len(sel), 0)),
                      eval_legendre(l, cosg) * ww)
            zeta[l] += wp[p] * (2 * l + 1) / (4 * math.pi) * acc
    return zeta


def zeta_sphere_pivots_triangles(x, y, z, w, nbins, theta_min, theta_max, mmax, h):
    """Shared pivots on the sphere: numpy grouping of the sphere's lattice points by pivot cells of
    Hq = max(1, floor(h scale)), pivots at the round-half-up mean, then the triangle form."""
    q, sc, T = sphere_lattice(x, y, z, nbins, theta_min, theta_max)
    w = np.ones(len(q)) if w is None else np.asarray(w, dtype=np.float64)
    Hq = max(1, int(math.floor(h * sc)))
    keys, inv = np.unique((q // Hq)[:, ::-1], axis=0, return_inverse=True)
    inv = inv.ravel()
    G = len(keys)
    cnt = np.bincount(inv, minlength=G).astype(np.int64)
    sums = np.zeros((G, 3), dtype=np.int64)
    np.add.at(sums, inv, q)
    W = np.zeros(G)
    np.add.at(W, inv, w)
    X = (2 * sums + cnt[:, None]) // (2 * cnt[:, None])
    zeta = np.zeros((mmax + 1, nbins, nbins))
    for g in range(G):
        sphere_triangles_at(X[g], W[g], -1, q, w, sc, T, nbins, mmax, zeta, None, None, g)
    return zeta, G

