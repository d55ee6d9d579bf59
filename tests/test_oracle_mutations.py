"""The pins are strong enough: each planted mistake in a copy of the oracle fails one of them.

Every mutant is a textual edit of ``oracle/tpcf_oracle.c`` compiled into a temporary library
on the CPU; the committed oracle is never modified.
"""
import ctypes
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import catalogs
import oracle
from tests import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "tpcf_oracle.c")

MUTANTS = {
    "normalisation 2l-1": ("(2.0L * l + 1.0L)", "(2.0L * l - 1.0L)"),
    "no Condon-Shortley phase": ("pmm *= -(2.0 * i - 1.0) * sx", "pmm *= (2.0 * i - 1.0) * sx"),
    "recurrence coefficient": ("(l + m - 1.0) * P[l - 2][m]", "(l + m + 1.0) * P[l - 2][m]"),
    "primary weight dropped": ("zacc[((size_t)l * nb + b1) * nb + b2] += wp * s;",
                               "zacc[((size_t)l * nb + b1) * nb + b2] += s;"),
    "lower edge exclusive": ("R2 < P->T[0] || R2 >= P->T[P->nbins]",
                             "R2 <= P->T[0] || R2 >= P->T[P->nbins]"),
    "inner edge inclusive": ("while (b + 1 < P->nbins && R2 >= P->T[b + 1]) b++;",
                             "while (b + 1 < P->nbins && R2 > P->T[b + 1]) b++;"),
    "no minimum image": ("if (d >= M / 2) d -= M;", "if (d >= M) d -= M;"),
    "missing conjugate in contraction": ("* conj(alm[(size_t)b2 * nc + c]));",
                                         "* alm[(size_t)b2 * nc + c]);"),
    "m = l term dropped": ("for (int m = -l; m <= l; m++) {", "for (int m = -l; m < l; m++) {"),
    "negative m phase": ("((m & 1) ? -1.0 : 1.0) * conj(y)", "conj(y)"),
    "secondary weight dropped": ("a[c] += P->w[j] * conj(Y[c]);", "a[c] += conj(Y[c]);"),
    "pair sums: primary weight dropped": ("dpart[c * nb + b] += w[p] * w[j];",
                                          "dpart[c * nb + b] += w[j];"),
    "edge correction: projection factor": ("M[L][l2] = 0.5 * (2.0 * L + 1.0) * s;",
                                           "M[L][l2] = 0.5 * (2.0 * l2 + 1.0) * s;"),
    "sphere: angle used as chord": ("const double v = 2.0 * sin(0.5 * th) * sc;",
                                    "const double v = th * sc;"),
    "sphere: second tangent vector": ("np_[0] * e1[1] - np_[1] * e1[0]};",
                                      "np_[0] * e1[1] + np_[1] * e1[0]};"),
    "sphere: no basis at the pole": ("if (l1 < 1e-6) { /* x x n */", "if (l1 < 0.0) { /* x x n */"),
    "sphere: primary weight dropped": ("+= wp * creal(am[b1 * M1 + m] * conj(am[b2 * M1 + m]));",
                                       "+= creal(am[b1 * M1 + m] * conj(am[b2 * M1 + m]));"),
    "pivots: mean rounded down": ("pq[ax * n + G] = (2 * sum[ax] + cnt) / (2 * cnt);",
                                  "pq[ax * n + G] = sum[ax] / cnt;"),
    "pivots: group weight is the mean": ("pw[G] = W;", "pw[G] = W / (double)cnt;"),
    "pivots: group key ignores y": ("keys[i].gy = q[n + i] / Hq;", "keys[i].gy = 0;"),
    "degenerate: w_j in place of w_j^2": ("part[c * nb + b] += P->w[p] * P->w[j] * P->w[j];",
                                          "part[c * nb + b] += P->w[p] * P->w[j];"),
    "degenerate: factor 2l - 1": ("D[l * nb + b] = (2.0 * l + 1.0) / (4.0 * 3.14159265358979323846) * S[b];",
                                  "D[l * nb + b] = (2.0 * l - 1.0) / (4.0 * 3.14159265358979323846) * S[b];"),
    "degenerate sphere: 3D factor": ("for (int b = 0; b < nb; b++) D[m * nb + b] = S[b];",
                                     "for (int b = 0; b < nb; b++) D[m * nb + b] = (2.0 * m + 1.0) * S[b];"),
    "edge correction: 8-node quadrature": ("enum { NQ = 32 };", "enum { NQ = 8 };"),
    "edge correction: 16-node quadrature": ("enum { NQ = 32 };", "enum { NQ = 16 };"),
    "sphere edge correction: 16-point trapezoid": ("enum { NQ = 64 };", "enum { NQ = 16 };"),
    "sphere edge correction: 32-point trapezoid": ("enum { NQ = 64 };", "enum { NQ = 32 };"),
    "sphere edge correction: weight of m' = 0": ("A[m][mp] = (mp == 0 ? 1.0 : 2.0) * t * (twopi / NQ);",
                                                 "A[m][mp] = 2.0 * t * (twopi / NQ);"),
}


def _pins():
    """Cheap versions of the pins; returns the names of the ones that fail."""
    failed = []
    # worked triangle
    O = np.array([125.0, 125.0, 125.0])
    Pt = np.array([O, O + [10.0, 0, 0], O + [0, 10.0, 0]])
    r = oracle.zeta(Pt[:, 0], Pt[:, 1], Pt[:, 2], None, 250.0, True, 10, 5.0, 50.0, 4)
    for l in range(5):
        c = (2 * l + 1) / (4 * math.pi)
        if (abs(r.zeta[l, 1, 1] - c * (4 + 2 * eval_legendre(l, 0.0))) > 1e-9
                or abs(r.zeta[l, 1, 2] - 2 * c * eval_legendre(l, 2**-0.5)) > 1e-9):
            failed.append("worked triangle")
            break
    # brute-force triangles, weighted, both geometries
    rng = np.random.default_rng(3)
    P = rng.random((70, 3)) * 50.0
    w = rng.normal(0.5, 1.0, 70)
    for periodic in (True, False):
        z = oracle.zeta(P[:, 0], P[:, 1], P[:, 2], w, 50.0, periodic, 4, 2.0, 20.0, 5).zeta
        ref = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, 50.0, periodic, 4, 2.0, 20.0, 5)
        if np.max(np.abs(z - ref)) > 1e-12 * np.max(np.abs(ref)):
            failed.append("brute-force triangles")
            break
    # degenerate (j = k) term: the brute-force j = k part, 3D and sphere
    D = oracle.degenerate(P[:, 0], P[:, 1], P[:, 2], w, 50.0, True, 4, 2.0, 20.0, 5)
    part = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, 50.0, True, 4, 2.0, 20.0, 5, drop_jk=True)
    full = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, 50.0, True, 4, 2.0, 20.0, 5)
    dd = np.array([np.diag(full[l] - part[l]) for l in range(6)])
    if np.max(np.abs(D - dd)) > 1e-12 * np.max(np.abs(dd)):
        failed.append("degenerate term")
    # Y_lm against scipy
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    Y = oracle.ylm(v[:, 0], v[:, 1], v[:, 2], 6)
    th, ph = np.arccos(v[:, 2]), np.arctan2(v[:, 1], v[:, 0])
    ok = all(np.allclose(Y[:, l * l + l + m], sph_harm_y(l, m, th, ph), atol=1e-13, rtol=0)
             for l in range(7) for m in range(-l, l + 1))
    if not ok:
        failed.append("Y_lm vs scipy")
    # exact bin edges
    box, K = 256.0, 27
    s = box / 2**K
    x0 = 100.0 + 0.5 * s
    xs = np.array([x0, x0 + 16.0, x0 + 16.0 - s, x0 + 64.0, x0 + 8.0])
    zz = np.full(5, 50.0 + 0.5 * s)
    r = oracle.zeta(xs, zz, zz, None, box, True, 7, 8.0, 64.0, 0, 0, 1, want_counts=True)
    if list(r.counts[0]) != [2, 1, 0, 0, 0, 0, 0]:
        failed.append("bin edges")
    # translation across the periodic boundary
    K = brute.lattice_bits(60.0, 20.0, True)
    M = 2**K
    q = rng.integers(0, M, size=(60, 3))
    X = (q + 0.5) * (60.0 / M)
    z0 = oracle.zeta(X[:, 0], X[:, 1], X[:, 2], w[:60], 60.0, True, 4, 2.0, 20.0, 3).zeta
    Xt = ((q + M // 2 + 12345) % M + 0.5) * (60.0 / M)
    z1 = oracle.zeta(Xt[:, 0], Xt[:, 1], Xt[:, 2], w[:60], 60.0, True, 4, 2.0, 20.0, 3).zeta
    if np.max(np.abs(z1 - z0)) > 1e-12 * np.max(np.abs(z0)):
        failed.append("translation")
    # two-point by-product against the pair table
    Pc = np.concatenate([P[:40], P[:3]])
    wc = np.concatenate([w[:40], w[:3]])
    n_o, d_o = oracle.pair_sums(Pc[:, 0], Pc[:, 1], Pc[:, 2], wc, 50.0, True, 4, 0.0, 20.0)
    n_b, d_b = brute.pair_sums(Pc[:, 0], Pc[:, 1], Pc[:, 2], wc, 50.0, True, 4, 0.0, 20.0)
    if not np.array_equal(n_o, n_b) or np.max(np.abs(d_o - d_b)) > 1e-12 * np.max(np.abs(d_b)):
        failed.append("pair sums")
    # edge correction at l_max = 2 against the hand-written squared-3j coupling matrix
    f1, f2 = 0.3, -0.2
    Re = np.zeros((3, 1, 1))
    Re[:, 0, 0] = [1.0, f1, f2]
    Me = np.array([[1.0, f1 / 3, f2 / 5], [f1, 3 * (1 / 3 + 2 * f2 / 15), 2 * f1 / 5],
                   [f2, 2 * f1 / 3, 1 + 2 * f2 / 7]])
    zt = np.array([0.7, -0.4, 0.25])
    if np.abs(oracle.edge_correct((Me @ zt)[:, None, None], Re)[:, 0, 0] - zt).max() > 1e-12:
        failed.append("edge correction")
    # sphere: basis-free triangle form, and the pivot at the pole
    ra = np.concatenate([1.0 + 0.15 * rng.standard_normal(40), rng.random(29) * 2 * np.pi, [0.0]])
    dec = np.concatenate([0.3 + 0.15 * rng.standard_normal(40), np.pi / 2 - 0.2 * rng.random(29),
                          [np.pi / 2]])
    ws = rng.normal(1.0, 0.5, 70)
    u = catalogs.radec_to_unit(ra, dec)
    zs = oracle.zeta_sphere(*u, ws, 4, 0.01, 0.3, 5).zeta
    ref, _, _ = brute.zeta_sphere_triangles(*u, ws, 4, 0.01, 0.3, 5)
    if not np.all(np.isfinite(zs)) or np.max(np.abs(zs - ref)) > 1e-12 * np.max(np.abs(ref)):
        failed.append("sphere triangles")
    Ds = oracle.degenerate_sphere(*u, ws - 1.0, 4, 0.01, 0.3, 5)
    fs, _, _ = brute.zeta_sphere_triangles(*u, ws - 1.0, 4, 0.01, 0.3, 5)
    ps, _, _ = brute.zeta_sphere_triangles(*u, ws - 1.0, 4, 0.01, 0.3, 5, drop_jk=True)
    dds = np.array([np.diag(fs[m] - ps[m]) for m in range(6)])
    if np.max(np.abs(Ds - dds)) > 1e-12 * np.max(np.abs(dds)):
        failed.append("sphere degenerate term")
    # sphere edge correction: N built from the closed-form coupling is solved back
    Rs = np.zeros((3, 1, 1))
    Rs[:, 0, 0] = [1.0, 0.25, -0.1]
    cs = np.array([0.6, -0.3, 0.2])
    Ns = np.zeros((3, 1, 1))
    Rk = lambda k: Rs[k, 0, 0] if k <= 2 else 0.0
    for m in range(3):
        Ns[m, 0, 0] = sum((1.0 if mp == 0 else 2.0) * 0.5 * (Rk(m + mp) + Rk(abs(m - mp))) * cs[mp] for mp in range(3))
    if np.abs(oracle.edge_correct_sphere(Ns, Rs)[:, 0, 0] - cs).max() > 1e-12:
        failed.append("sphere edge correction")
    # edge corrections at the oracle's highest order (16), against closed forms that use neither
    # quadrature nor 3j symbols: Legendre-series and cosine-series products
    from tests.test_oracle_pins import _tridiagonal_3d, _tridiagonal_sphere
    Lh = 16
    Rh = np.zeros((Lh + 1, 1, 1))
    Rh[:, 0, 0] = 0.2 * rng.normal(size=Lh + 1) / np.arange(1, Lh + 2)
    Rh[0, 0, 0] = 1.5
    zh = rng.normal(size=Lh + 1)
    Nh = np.polynomial.legendre.legmul(zh, Rh[:, 0, 0])[: Lh + 1][:, None, None]
    if np.abs(oracle.edge_correct(Nh, Rh)[:, 0, 0] - zh).max() > 1e-10:
        failed.append("edge correction, order 16")
    Nt = (1.5 * _tridiagonal_3d(10, 0.4) @ zh[:11])[:, None, None]
    Rt = np.zeros((11, 1, 1))
    Rt[0, 0, 0], Rt[1, 0, 0] = 1.5, 0.6
    if np.abs(oracle.edge_correct(Nt, Rt)[:, 0, 0] - zh[:11]).max() > 1e-10:
        failed.append("edge correction, order 10")
    two = lambda v: np.concatenate([v[:0:-1], v])
    Nsh = np.convolve(two(zh), two(Rh[:, 0, 0]))[2 * Lh: 3 * Lh + 1][:, None, None]
    if np.abs(oracle.edge_correct_sphere(Nsh, Rh)[:, 0, 0] - zh).max() > 1e-10:
        failed.append("sphere edge correction, order 16")
    Nst = (1.5 * _tridiagonal_sphere(10, 0.3) @ zh[:11])[:, None, None]
    Rst = np.zeros((11, 1, 1))
    Rst[0, 0, 0], Rst[1, 0, 0] = 1.5, 0.45
    if np.abs(oracle.edge_correct_sphere(Nst, Rst)[:, 0, 0] - zh[:11]).max() > 1e-10:
        failed.append("sphere edge correction, order 10")
    # shared pivots: group pivots and zeta against the numpy grouping and Legendre form
    cP = (rng.random((4, 3))[rng.integers(0, 4, 150)] * 40.0 + rng.normal(0, 2.0, (150, 3))) % 40.0
    cw = rng.normal(1.0, 0.4, 150)
    rp = oracle.zeta_pivots(cP[:, 0], cP[:, 1], cP[:, 2], cw, 40.0, True, 4, 1.0, 10.0, 3, 2.5)
    X, W, q, K = brute.pivot_groups(cP[:, 0], cP[:, 1], cP[:, 2], cw, 40.0, True, 10.0, 2.5)
    ok = rp.ngroups == len(X) and np.array_equal(rp.gq, X) and np.allclose(rp.gw, W, rtol=0, atol=1e-13)
    if ok:
        ref = brute.zeta_triangles_lattice(X, W, q, cw, K, True, brute.thresholds(4, 1.0, 10.0, 40.0, K), 4, 3)
        ok = np.max(np.abs(rp.zeta - ref)) <= 1e-12 * np.max(np.abs(ref))
    if not ok:
        failed.append("shared pivots")
    return failed


@pytest.fixture
def mutant_loader(monkeypatch):
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")

    def load(old, new):
        src = open(SRC).read()
        assert src.count(old) == 1, old
        path_c = os.path.join(tmp, "mut.c")
        open(path_c, "w").write(src.replace(old, new))
        so = os.path.join(tmp, "mut%d.so" % len(os.listdir(tmp)))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so,
                               path_c, "-lm"])
        monkeypatch.setattr(oracle, "_LIB", so)
        monkeypatch.setattr(oracle, "build", lambda force=False: so)
        monkeypatch.setattr(oracle, "_lib", None)

    yield load
    oracle._lib = None
    shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_oracle_passes_cheap_pins():
    assert _pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_loader):
    old, new = MUTANTS[name]
    mutant_loader(old, new)
    failed = _pins()
    assert failed, f"mutant '{name}' passed every pin"
