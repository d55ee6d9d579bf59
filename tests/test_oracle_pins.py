"""Pins for the FP64 oracle: each test checks it against something other than itself.

* worked triangle: hand-derived closed form (golden fixture);
* brute-force triangle sum in the Legendre form (no Y_lm, independent numpy route);
* l = 0 reduces to products of pair counts;
* Y_lm against scipy's spherical harmonics and its special values;
* the 48 cube symmetries and lattice translations (exact on the lattice);
* Poisson expectation on uniform boxes;
* positive semi-definiteness, bin merging, weight homogeneity, primary-range additivity;
* integer pair counts against a numpy pair loop, including pairs exactly on bin edges.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import catalogs
import oracle
from tests import brute

HERE = os.path.dirname(os.path.abspath(__file__))


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------- worked example

def _worked_points():
    O = np.array([125.0, 125.0, 125.0])
    P = np.array([O, O + [10.0, 0, 0], O + [0, 10.0, 0]])
    return P[:, 0], P[:, 1], P[:, 2]


def test_worked_triangle_fixture_matches_closed_form():
    rows = np.loadtxt(os.path.join(HERE, "golden", "worked_triangle.txt"))
    for l, z11, z22, z12 in rows:
        l = int(l)
        c = (2 * l + 1) / (4 * math.pi)
        assert z11 == pytest.approx(c * (4 + 2 * eval_legendre(l, 0.0)), abs=1e-9)
        assert z22 == pytest.approx(2 * c, abs=1e-9)
        assert z12 == pytest.approx(2 * c * eval_legendre(l, 1 / math.sqrt(2)), abs=1e-9)


def test_worked_triangle():
    x, y, z = _worked_points()
    r = oracle.zeta(x, y, z, None, 250.0, True, 10, 5.0, 50.0, 4, want_counts=True)
    rows = np.loadtxt(os.path.join(HERE, "golden", "worked_triangle.txt"))
    expect = np.zeros((5, 10, 10))
    for l, z11, z22, z12 in rows:
        l = int(l)
        expect[l, 1, 1], expect[l, 2, 2] = z11, z22
        expect[l, 1, 2] = expect[l, 2, 1] = z12
    np.testing.assert_allclose(r.zeta, expect, atol=5e-10)
    cnt = np.zeros((3, 10), dtype=np.int64)
    cnt[0, 1] = 2
    cnt[1, 1] = cnt[1, 2] = cnt[2, 1] = cnt[2, 2] = 1
    np.testing.assert_array_equal(r.counts, cnt)
    assert r.npairs == 6


# ---------------------------------------------------------------- brute-force triangles

@pytest.mark.parametrize("periodic", [True, False])
def test_bruteforce_triangles(periodic):
    rng = np.random.default_rng(7)
    n, box = 160, 100.0
    P = rng.random((n, 3)) * box
    w = rng.normal(0.3, 1.0, n)  # includes negative weights
    nb, rmin, rmax, lmax = 6, 4.0, 40.0, 6
    r = oracle.zeta(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax)
    ref = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax)
    for l in range(lmax + 1):
        assert _rel(r.zeta[l], ref[l]) < 1e-12, l


def test_bruteforce_triangles_subset_at_larger_n():
    c = catalogs.uniform(1500, 120.0, 3)
    w = catalogs.gaussian_weights(c.n, 4)
    prim = [5, 77, 1020]
    nb, rmin, rmax, lmax = 5, 3.0, 25.0, 8
    ref = brute.zeta_triangles(c.x, c.y, c.z, w, c.box, True, nb, rmin, rmax, lmax, primaries=prim)
    tot = np.zeros_like(ref)
    for p in prim:
        tot += oracle.zeta(c.x, c.y, c.z, w, c.box, True, nb, rmin, rmax, lmax, p, p + 1).zeta
    for l in range(lmax + 1):
        assert _rel(tot[l], ref[l]) < 1e-12


# ---------------------------------------------------------------- the degenerate (j = k) term

def test_degenerate_worked_triangle():
    """The three-point example: bin 1 holds A and B for O, and O for A and for B (4 secondaries,
    unit weights); bin 2 holds B for A and A for B (2). D_l = (2l+1)/(4 pi) x those counts, and
    on bin 2, where no primary has two secondaries, D_l(2) is all of zeta_l(2, 2)."""
    x, y, z = np.array([125.0, 135.0, 125.0]), np.array([125.0, 125.0, 135.0]), np.full(3, 125.0)
    D = oracle.degenerate(x, y, z, None, 250.0, True, 10, 5.0, 50.0, 4)
    c = np.array([(2 * l + 1) / (4 * math.pi) for l in range(5)])
    expect = np.zeros((5, 10))
    expect[:, 1] = 4 * c
    expect[:, 2] = 2 * c
    np.testing.assert_allclose(D, expect, rtol=1e-15, atol=0)
    zt = oracle.zeta(x, y, z, None, 250.0, True, 10, 5.0, 50.0, 4).zeta
    np.testing.assert_allclose(D[:, 2], zt[:, 2, 2], rtol=1e-14)


@pytest.mark.parametrize("periodic", [True, False])
def test_degenerate_is_the_jk_part_of_brute_force(periodic):
    """zeta with every (j, k) minus zeta without j = k (both from the brute-force triangle form)
    is D_l(b) on the diagonal and zero off it; signed weights, so w_j^2 against w_j matters."""
    rng = np.random.default_rng(17)
    n, box = 140, 100.0
    P = rng.random((n, 3)) * box
    w = rng.normal(0.2, 1.0, n)
    nb, rmin, rmax, lmax = 6, 4.0, 40.0, 5
    full = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax)
    part = brute.zeta_triangles(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax, drop_jk=True)
    D = oracle.degenerate(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax)
    diff = full - part
    for l in range(lmax + 1):
        np.testing.assert_allclose(np.diag(diff[l]), D[l], rtol=1e-11, atol=1e-12 * np.abs(D[l]).max())
        assert np.abs(diff[l] - np.diag(np.diag(diff[l]))).max() <= 1e-12 * np.abs(D[l]).max()
    # weight homogeneity: w -> a w scales D by a^3; primary ranges add up
    D2 = oracle.degenerate(P[:, 0], P[:, 1], P[:, 2], -2.0 * w, box, periodic, nb, rmin, rmax, lmax)
    np.testing.assert_allclose(D2, -8.0 * D, rtol=1e-14)
    Da = oracle.degenerate(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax, 0, 50)
    Db = oracle.degenerate(P[:, 0], P[:, 1], P[:, 2], w, box, periodic, nb, rmin, rmax, lmax, 50, n)
    np.testing.assert_allclose(Da + Db, D, rtol=1e-13, atol=1e-14 * np.abs(D).max())


def test_degenerate_sphere_is_the_jk_part_of_brute_force():
    """On the sphere |exp(-i m phi)|^2 = 1: D_m(b) does not depend on m and equals the diagonal
    of the brute-force zeta_m minus its j != k part."""
    x, y, z, w = _sphere_points(150, 4)
    w = w - 1.0
    full, _, _ = brute.zeta_sphere_triangles(x, y, z, w, 5, 0.01, 0.3, 6)
    part, _, _ = brute.zeta_sphere_triangles(x, y, z, w, 5, 0.01, 0.3, 6, drop_jk=True)
    D = oracle.degenerate_sphere(x, y, z, w, 5, 0.01, 0.3, 6)
    assert np.abs(D).max() > 0
    for m in range(7):
        np.testing.assert_allclose(np.diag(full[m] - part[m]), D[m], rtol=1e-11, atol=1e-12 * np.abs(D).max())
        np.testing.assert_array_equal(D[m], D[0])


# ---------------------------------------------------------------- l = 0 and pair counts

def test_l0_is_product_of_pair_counts():
    c = catalogs.uniform(400, 80.0, 11)
    w = catalogs.gaussian_weights(c.n, 12, 1.0, 0.5)
    nb, rmin, rmax = 8, 2.0, 30.0
    r = oracle.zeta(c.x, c.y, c.z, w, c.box, True, nb, rmin, rmax, 2)
    Np = np.zeros((c.n, nb))
    for p, j, b, u in brute.pair_table(c.x, c.y, c.z, c.box, True, nb, rmin, rmax):
        Np[p, b] += w[j]
    ref = np.einsum("p,pa,pb->ab", w, Np, Np) / (4 * math.pi)
    assert _rel(r.zeta[0], ref) < 1e-12


@pytest.mark.parametrize("periodic", [True, False])
def test_pair_counts_exact(periodic):
    c = catalogs.uniform(300, 60.0, 21)
    nb, rmin, rmax = 7, 1.5, 22.0
    r = oracle.zeta(c.x, c.y, c.z, None, c.box, periodic, nb, rmin, rmax, 1, want_counts=True)
    ref = brute.pair_counts(c.x, c.y, c.z, c.box, periodic, nb, rmin, rmax)
    np.testing.assert_array_equal(r.counts, ref)
    assert r.npairs == int(ref.sum())


@pytest.mark.parametrize("periodic", [True, False])
def test_pair_sums_against_brute_force(periodic):
    """The two-point by-product: ordered pairs per bin (exact) and sum of w_p w_j per bin,
    against an independent numpy pair table; unit weights give dd == npairs; the totals agree
    with the multipole oracle's pair count; every unordered pair counts twice."""
    c = catalogs.lognormal(350, 70.0, 61, grid=16)
    w = catalogs.gaussian_weights(c.n, 62, 1.0, 0.7)
    nb, rmin, rmax = 6, 2.0, 25.0
    npairs, dd = oracle.pair_sums(c.x, c.y, c.z, w, c.box, periodic, nb, rmin, rmax)
    bn, bdd = brute.pair_sums(c.x, c.y, c.z, w, c.box, periodic, nb, rmin, rmax)
    np.testing.assert_array_equal(npairs, bn)
    assert _rel(dd, bdd) < 1e-13
    assert np.all(npairs % 2 == 0)
    n1, d1 = oracle.pair_sums(c.x, c.y, c.z, None, c.box, periodic, nb, rmin, rmax)
    np.testing.assert_array_equal(n1, npairs)
    np.testing.assert_array_equal(d1, npairs.astype(float))
    assert oracle.zeta(c.x, c.y, c.z, w, c.box, periodic, nb, rmin, rmax, 0).npairs == int(npairs.sum())
    # primary ranges add up
    a = oracle.pair_sums(c.x, c.y, c.z, w, c.box, periodic, nb, rmin, rmax, 0, 100)
    b = oracle.pair_sums(c.x, c.y, c.z, w, c.box, periodic, nb, rmin, rmax, 100, c.n)
    np.testing.assert_array_equal(a[0] + b[0], npairs)
    assert _rel(a[1] + b[1], dd) < 1e-13


def test_edge_correction_closed_forms():
    """Edge correction (zeta solves M(R) zeta = N / R_0): an isotropic R gives N / R_0; at
    l_max = 2 the coupling matrix written out from the standard values of the squared 3j
    symbols, (0 1 1) = 1/3, (0 2 2) = 1/5, (1 1 2) = 2/15, (2 2 2) = 2/35, inverts a known
    zeta; scaling N and R scales zeta by their ratio; catalogues are independent."""
    rng = np.random.default_rng(5)
    R = np.zeros((4, 3, 3))
    R[0] = rng.uniform(1.0, 3.0, (3, 3))
    N = rng.normal(size=(4, 3, 3))
    assert _rel(oracle.edge_correct(N, R), N / R[0]) < 1e-14
    f1, f2 = 0.3, -0.2
    R = np.zeros((3, 1, 1))
    R[:, 0, 0] = [2.0, 2.0 * f1, 2.0 * f2]
    M = np.array([[1.0, f1 / 3, f2 / 5],
                  [f1, 3 * (1 / 3 + 2 * f2 / 15), 3 * 2 * f1 / 15],
                  [f2, 5 * 2 * f1 / 15, 5 * (1 / 5 + 2 * f2 / 35)]])
    zt = np.array([0.7, -0.4, 0.25])
    N = (2.0 * M @ zt)[:, None, None]
    assert np.abs(oracle.edge_correct(N, R)[:, 0, 0] - zt).max() < 1e-14
    # scaling and batches
    R = np.concatenate([R, R], axis=1).repeat(2, axis=2)
    R[1:] *= 0.5
    N = rng.normal(size=R.shape)
    z = oracle.edge_correct(N, R)
    assert _rel(oracle.edge_correct(3.0 * N, 2.0 * R), 1.5 * z) < 1e-13
    zb = oracle.edge_correct(np.stack([N, 2 * N]), np.stack([R, R]))
    assert _rel(zb[0], z) < 1e-15 and _rel(zb[1], 2 * z) < 1e-14
    # bin pairs without randoms give 0
    R0 = R.copy()
    R0[:, 0, 1] = 0.0
    assert not oracle.edge_correct(N, R0)[:, 0, 1].any()


def _tridiagonal_3d(lmax, a):
    """Coupling matrix for R(mu) = R_0 (1 + a P_1(mu)), from mu P_l = ((l+1) P_{l+1} + l P_{l-1}) / (2l+1):
    the Legendre coefficient L of P_l(mu) (1 + a mu) is delta_{lL} + a (l+1)/(2l+1) delta_{L,l+1}
    + a l/(2l+1) delta_{L,l-1}."""
    M = np.eye(lmax + 1)
    for l in range(lmax + 1):
        if l + 1 <= lmax:
            M[l + 1, l] += a * (l + 1) / (2 * l + 1)
        if l >= 1:
            M[l - 1, l] += a * l / (2 * l + 1)
    return M


@pytest.mark.parametrize("lmax", [10, 16])
def test_edge_correction_high_order(lmax):
    """Edge correction at the orders the library runs (l_max = 10) and at the oracle's cap (16),
    pinned without 3j symbols or quadrature: (1) with R(mu) = R_0 (1 + a P_1(mu)) the coupling
    matrix is I plus the tridiagonal of the three-term recurrence of mu P_l; N = R_0 M zeta is
    solved back; (2) for random Legendre series zeta(mu) and R(mu), N(mu) = zeta(mu) R(mu) is
    their product taken with numpy's Legendre-series multiplication (exact, degree 2 l_max)
    truncated at l_max, and zeta is recovered."""
    rng = np.random.default_rng(100 + lmax)
    R0, a = 2.5, 0.45
    zt = rng.normal(size=lmax + 1)
    R = np.zeros((lmax + 1, 1, 1))
    R[0, 0, 0], R[1, 0, 0] = R0, a * R0
    N = (R0 * _tridiagonal_3d(lmax, a) @ zt)[:, None, None]
    assert np.abs(oracle.edge_correct(N, R)[:, 0, 0] - zt).max() < 1e-12 * np.abs(zt).max()
    # random series, several bin pairs at once
    nb = 3
    Rr = np.zeros((lmax + 1, nb, nb))
    Rr[0] = rng.uniform(1.0, 2.0, (nb, nb))
    Rr[1:] = 0.25 * rng.normal(size=(lmax, nb, nb)) * Rr[0] / np.arange(1, lmax + 1)[:, None, None]
    zr = rng.normal(size=(lmax + 1, nb, nb))
    Nr = np.zeros_like(zr)
    for i in range(nb):
        for j in range(nb):
            Nr[:, i, j] = np.polynomial.legendre.legmul(zr[:, i, j], Rr[:, i, j])[: lmax + 1]
    assert np.abs(oracle.edge_correct(Nr, Rr) - zr).max() < 1e-11 * np.abs(zr).max()


def test_bin_edges_are_half_open():
    # box 256 and bins [8, 64) of width 8: with K = 27 every edge is a whole number of lattice
    # steps, so separations can sit exactly on an edge. A separation of exactly 16 belongs to
    # bin 1 ([16, 24)); one lattice step less belongs to bin 0; exactly 8 is bin 0; exactly 64
    # is out of range.
    box, nb, rmin, rmax = 256.0, 7, 8.0, 64.0
    K = oracle.lattice_bits(box, rmax, True)
    assert K == 27
    s = box / 2**K
    x0 = 100.0 + 0.5 * s  # mid-cell so snapping is unambiguous
    xs = np.array([x0, x0 + 16.0, x0 + 16.0 - s, x0 + 64.0, x0 + 8.0])
    zeros = np.full(5, 50.0 + 0.5 * s)
    r = oracle.zeta(xs, zeros, zeros, None, box, True, nb, rmin, rmax, 0, 0, 1, want_counts=True)
    np.testing.assert_array_equal(r.counts[0], [2, 1, 0, 0, 0, 0, 0])
    T = oracle.thresholds(nb, rmin, rmax, box, K)
    assert int(T[1]) == (16 * 2**K // 256) ** 2
    assert int(T[0]) == (8 * 2**K // 256) ** 2 and int(T[7]) == (64 * 2**K // 256) ** 2
    assert [int(t) for t in T] == [int(v) for v in brute.thresholds(nb, rmin, rmax, box, K)]


# ---------------------------------------------------------------- spherical harmonics

def test_ylm_against_scipy():
    rng = np.random.default_rng(5)
    v = rng.normal(size=(4000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    lmax = 10
    Y = oracle.ylm(v[:, 0], v[:, 1], v[:, 2], lmax)
    theta = np.arccos(np.clip(v[:, 2], -1, 1))
    phi = np.arctan2(v[:, 1], v[:, 0])
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            ref = sph_harm_y(l, m, theta, phi)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13, rtol=0)


def test_ylm_special_values():
    lmax = 12
    Y = oracle.ylm(np.array([0.0, 0.0]), np.array([0.0, 0.0]), np.array([1.0, -1.0]), lmax)
    assert Y[0, 0] == pytest.approx(1 / math.sqrt(4 * math.pi), abs=1e-15)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            c = l * l + l + m
            if m == 0:
                val = math.sqrt((2 * l + 1) / (4 * math.pi))
                assert Y[0, c] == pytest.approx(val, abs=1e-13)
                assert Y[1, c] == pytest.approx(val * (-1) ** l, abs=1e-13)
            else:
                assert abs(Y[0, c]) < 1e-13 and abs(Y[1, c]) < 1e-13
    # Y_11 on the x axis: -sqrt(3/(8 pi)) (Condon-Shortley phase)
    Y = oracle.ylm(np.array([1.0]), np.array([0.0]), np.array([0.0]), 1)
    assert Y[0, 3].real == pytest.approx(-math.sqrt(3 / (8 * math.pi)), abs=1e-15)


# ---------------------------------------------------------------- invariances

def _lattice_catalog(n, box, rmax, seed, periodic=True):
    """Points exactly at lattice-cell centres, so symmetries act exactly on the lattice."""
    K = oracle.lattice_bits(box, rmax, periodic)
    rng = np.random.default_rng(seed)
    q = rng.integers(0, 2**K, size=(n, 3))
    return q, K


def _from_lattice(q, box, K):
    return (q.astype(np.float64) + 0.5) * (box / 2**K)


def test_cube_symmetries_periodic():
    box, nb, rmin, rmax, lmax = 60.0, 5, 2.0, 20.0, 6
    q, K = _lattice_catalog(250, box, rmax, 31)
    M = 2**K
    w = catalogs.gaussian_weights(250, 32)
    X = _from_lattice(q, box, K)
    base = oracle.zeta(X[:, 0], X[:, 1], X[:, 2], w, box, True, nb, rmin, rmax, lmax).zeta
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            qq = q[:, perm].copy()
            for a in range(3):
                if signs[a] < 0:
                    qq[:, a] = (M - 1 - qq[:, a]) % M  # reflection of cell centres
            Xs = _from_lattice(qq, box, K)
            z = oracle.zeta(Xs[:, 0], Xs[:, 1], Xs[:, 2], w, box, True, nb, rmin, rmax, lmax).zeta
            assert _rel(z, base) < 1e-12, (perm, signs)


def test_translation_and_permutation_invariance():
    box, nb, rmin, rmax, lmax = 60.0, 5, 2.0, 20.0, 5
    q, K = _lattice_catalog(250, box, rmax, 41)
    M = 2**K
    w = catalogs.gaussian_weights(250, 42)
    X = _from_lattice(q, box, K)
    base = oracle.zeta(X[:, 0], X[:, 1], X[:, 2], w, box, True, nb, rmin, rmax, lmax).zeta
    rng = np.random.default_rng(43)
    for _ in range(3):
        t = rng.integers(0, M, size=3)
        Xt = _from_lattice((q + t) % M, box, K)
        z = oracle.zeta(Xt[:, 0], Xt[:, 1], Xt[:, 2], w, box, True, nb, rmin, rmax, lmax).zeta
        assert _rel(z, base) < 1e-12
    # positions outside [0, L) wrap onto the same lattice
    Xw = X + box * np.array([1.0, -2.0, 3.0])
    z = oracle.zeta(Xw[:, 0], Xw[:, 1], Xw[:, 2], w, box, True, nb, rmin, rmax, lmax).zeta
    assert _rel(z, base) < 1e-12
    perm = rng.permutation(250)
    z = oracle.zeta(X[perm, 0], X[perm, 1], X[perm, 2], w[perm], box, True, nb, rmin, rmax,
                    lmax).zeta
    assert _rel(z, base) < 1e-12


def test_rotation_nonperiodic_with_tolerance():
    # Away from the walls a non-periodic catalogue's zeta is rotation invariant up to pairs
    # that move across a bin edge under the rotation (none for this configuration).
    rng = np.random.default_rng(51)
    n, box, nb, rmin, rmax, lmax = 200, 100.0, 4, 3.0, 15.0, 6
    P = 50.0 + (rng.random((n, 3)) - 0.5) * 40.0
    w = rng.normal(1.0, 0.3, n)
    A = rng.normal(size=(3, 3))
    Qm, _ = np.linalg.qr(A)
    Pr = (P - 50.0) @ Qm.T + 50.0
    z0 = oracle.zeta(P[:, 0], P[:, 1], P[:, 2], w, box, False, nb, rmin, rmax, lmax, want_counts=True)
    z1 = oracle.zeta(Pr[:, 0], Pr[:, 1], Pr[:, 2], w, box, False, nb, rmin, rmax, lmax, want_counts=True)
    np.testing.assert_array_equal(z0.counts, z1.counts)
    for l in range(lmax + 1):
        assert _rel(z1.zeta[l], z0.zeta[l]) < 1e-6


# ---------------------------------------------------------------- Poisson expectation

def _shell_fraction(box, rmin, rmax, nb):
    e = rmin + (rmax - rmin) / nb * np.arange(nb + 1)
    e[-1] = rmax
    return 4 * math.pi / 3 * (e[1:] ** 3 - e[:-1] ** 3) / box**3


@pytest.mark.slow
def test_poisson_expectation_uniform_box():
    N, box, nb, rmin, rmax, lmax = 10000, 250.0, 10, 5.0, 50.0, 4
    samples = []
    for seed in range(16):
        c = catalogs.uniform(N, box, seed)
        samples.append(oracle.zeta_catalog(c, nb, rmin, rmax, lmax).zeta)
    S = np.array(samples)
    mean = S.mean(0)
    se = S.std(0, ddof=1) / math.sqrt(len(samples))
    q = _shell_fraction(box, rmin, rmax, nb)
    E = np.zeros((lmax + 1, nb, nb))
    for l in range(lmax + 1):
        cl = (2 * l + 1) / (4 * math.pi)
        E[l] = cl * N * np.diag((N - 1) * q)
        if l == 0:
            E[l] += cl * N * (N - 1) * (N - 2) * np.outer(q, q)
    # the values quoted for this configuration
    assert E[0, 0, 0] == pytest.approx(4628.89, abs=0.01)
    assert E[0, 9, 9] == pytest.approx(5490719.27, abs=0.01)
    assert E[0, 0, 9] == pytest.approx(128982.96, abs=0.01)
    z = (mean - E) / se
    tested = np.zeros_like(z, dtype=bool)
    tested[0] = True
    for l in range(1, lmax + 1):
        tested[l] = np.eye(nb, dtype=bool)
    assert np.max(np.abs(z[tested])) < 6.0
    assert np.mean(z[tested] ** 2) < 2.0
    # relative agreement of the large entries
    assert np.max(np.abs(mean[0] - E[0]) / E[0]) < 0.01


# ---------------------------------------------------------------- structure

def test_psd_for_nonnegative_weights():
    c = catalogs.uniform(600, 70.0, 61)
    w = np.abs(catalogs.gaussian_weights(c.n, 62, 1.0, 0.4))
    z = oracle.zeta(c.x, c.y, c.z, w, c.box, True, 8, 2.0, 25.0, 8).zeta
    for l in range(z.shape[0]):
        np.testing.assert_allclose(z[l], z[l].T, rtol=0, atol=1e-12 * np.abs(z[l]).max())
        ev = np.linalg.eigvalsh(z[l])
        assert ev.min() >= -1e-12 * np.abs(ev).max()


def test_bin_merging():
    c = catalogs.uniform(500, 70.0, 71)
    w = catalogs.gaussian_weights(c.n, 72)
    z20 = oracle.zeta(c.x, c.y, c.z, w, c.box, True, 20, 2.0, 25.0, 6).zeta
    z1 = oracle.zeta(c.x, c.y, c.z, w, c.box, True, 1, 2.0, 25.0, 6).zeta
    np.testing.assert_allclose(z20.sum(axis=(1, 2)), z1[:, 0, 0], rtol=1e-12)


def test_weight_homogeneity_and_range_additivity():
    c = catalogs.uniform(400, 70.0, 81)
    w = catalogs.gaussian_weights(c.n, 82)
    args = (c.box, True, 6, 2.0, 25.0, 5)
    z = oracle.zeta(c.x, c.y, c.z, w, *args).zeta
    for alpha in (-1.0, 2.5):
        za = oracle.zeta(c.x, c.y, c.z, alpha * w, *args).zeta
        np.testing.assert_allclose(za, alpha**3 * z, rtol=1e-12, atol=1e-12 * np.abs(z).max())
    k = 137
    zlo = oracle.zeta(c.x, c.y, c.z, w, *args, p_begin=0, p_end=k).zeta
    zhi = oracle.zeta(c.x, c.y, c.z, w, *args, p_begin=k, p_end=c.n).zeta
    np.testing.assert_allclose(zlo + zhi, z, rtol=1e-12, atol=1e-13 * np.abs(z).max())


def test_degenerate_sizes():
    z = oracle.zeta(np.zeros(0), np.zeros(0), np.zeros(0), None, 10.0, True, 3, 1.0, 4.0, 2)
    assert z.zeta.shape == (3, 3, 3) and not z.zeta.any() and z.npairs == 0
    z = oracle.zeta(np.array([1.0]), np.array([1.0]), np.array([1.0]), None, 10.0, True, 3, 1.0, 4.0, 2)
    assert not z.zeta.any() and z.npairs == 0
    # two coincident points: no direction, no pair even with r_min = 0
    z = oracle.zeta(np.array([1.0, 1.0]), np.array([1.0, 1.0]), np.array([1.0, 1.0]), None, 10.0,
                    True, 3, 0.0, 4.0, 2)
    assert z.npairs == 0


# ---------------------------------------------------------------- projected fields on the sphere

def _sphere_points(n, seed):
    """A clustered cap, a polar cap (tangent basis switches near the pole) and the exact pole;
    unit vectors (x, y, z) and weights."""
    rng = np.random.default_rng(seed)
    h = n // 2
    ra = np.concatenate([1.0 + 0.15 * rng.standard_normal(h), rng.random(n - h - 1) * 2 * np.pi, [0.0]])
    dec = np.concatenate([0.3 + 0.15 * rng.standard_normal(h), np.pi / 2 - 0.2 * rng.random(n - h - 1),
                          [np.pi / 2]])
    return (*catalogs.radec_to_unit(ra, dec), rng.normal(1.0, 0.5, n))


def test_sphere_bruteforce_triangles():
    """zeta_m against the basis-free triangle form (cos of the angle between tangent-plane
    projections, no atan2 and no tangent basis); per-primary counts exact."""
    x, y, z, w = _sphere_points(160, 1)
    r = oracle.zeta_sphere(x, y, z, w, 5, 0.01, 0.3, 8, want_counts=True)
    zb, c, _ = brute.zeta_sphere_triangles(x, y, z, w, 5, 0.01, 0.3, 8)
    assert r.npairs > 5000
    assert np.array_equal(r.counts, c)
    assert _rel(r.zeta, zb) < 1e-12


def test_sphere_worked_example_at_the_pole():
    """Pivot at the north pole, three secondaries at colatitude 0.12 and position angles 0,
    2pi/3, 4pi/3 (bin 1 of [0.05, 0.25) in 4 bins) and one at colatitude 0.22, angle 0.5 (bin 3):
    zeta_m(1,1) = |sum_j exp(-i m phi_j)|^2 = 9 if 3 | m else 0,
    zeta_m(1,3) = sum_j cos(m (phi_j - 0.5)), zeta_m(3,3) = 1."""
    ang = np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3])
    ra = np.concatenate([[0.0], ang, [0.5]])
    dec = np.pi / 2 - np.array([0.0, 0.12, 0.12, 0.12, 0.22])
    r = oracle.zeta_sphere(*catalogs.radec_to_unit(ra, dec), None, 4, 0.05, 0.25, 7, 0, 1, want_counts=True)
    assert list(r.counts[0]) == [0, 3, 0, 1]
    for m in range(8):
        assert abs(r.zeta[m, 1, 1] - (9.0 if m % 3 == 0 else 0.0)) < 1e-6
        c13 = np.sum(np.cos(m * (ang - 0.5)))
        assert abs(r.zeta[m, 1, 3] - c13) < 1e-6 and abs(r.zeta[m, 3, 1] - c13) < 1e-6
        assert abs(r.zeta[m, 3, 3] - 1.0) < 1e-12
        assert np.all(r.zeta[m, [0, 2], :] == 0.0)


def test_sphere_m0_is_product_of_pair_sums():
    """zeta_0(b1, b2) = sum_p w_p S_p(b1) S_p(b2) with S_p(b) = sum_{j in b} w_j taken from the
    numpy pair table; with unit weights the integer pair counts, exactly."""
    x, y, z, w = _sphere_points(200, 2)
    r = oracle.zeta_sphere(x, y, z, None, 6, 0.0, 0.4, 2, want_counts=True)
    c = r.counts.astype(np.float64)
    assert np.array_equal(r.zeta[0], c.T @ c)
    _, _, S = brute.zeta_sphere_triangles(x, y, z, w, 6, 0.0, 0.4, 0)
    rw = oracle.zeta_sphere(x, y, z, w, 6, 0.0, 0.4, 0)
    assert _rel(rw.zeta[0], np.einsum("p,pa,pb->ab", w, S, S)) < 1e-12


def test_sphere_rotation_invariance():
    """A rigid rotation of the sphere changes every tangent basis but not zeta_m (up to the
    lattice snapping of the rotated points)."""
    x, y, z, w = _sphere_points(160, 3)
    v = np.stack([x, y, z], 1)
    Q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(3, 3)))
    u = v @ Q.T
    z0 = oracle.zeta_sphere(x, y, z, w, 5, 0.01, 0.3, 8)
    z1 = oracle.zeta_sphere(u[:, 0], u[:, 1], u[:, 2], w, 5, 0.01, 0.3, 8)
    assert z0.npairs == z1.npairs
    assert _rel(z1.zeta, z0.zeta) < 1e-6


def test_sphere_degenerate_and_invalid():
    e = np.zeros(0)
    r = oracle.zeta_sphere(e, e, e, None, 3, 0.0, 0.1, 4)
    assert r.npairs == 0 and not r.zeta.any()
    r = oracle.zeta_sphere(*catalogs.radec_to_unit(np.array([0.3]), np.array([0.2])), None, 3, 0.0, 0.1, 4)
    assert r.npairs == 0 and not r.zeta.any()
    # antipodal pair at the largest angle: in range only below theta_max = pi
    one, zero = np.array([1.0, -1.0]), np.zeros(2)
    r = oracle.zeta_sphere(one, zero, zero, None, 2, 0.0, np.pi, 1)
    assert r.npairs == 0
    r = oracle.zeta_sphere(*catalogs.radec_to_unit(np.array([0.0, 3.0]), zero), None, 2, 0.0, np.pi, 1)
    assert r.npairs == 2 and r.zeta[0, 1, 1] == 2.0
    for bad in [(3, 0.2, 0.1, 4), (0, 0.0, 0.1, 4), (3, 0.0, 4.0, 4), (3, 0.0, 0.1, -1)]:
        with pytest.raises(ValueError):
            oracle.zeta_sphere(one, zero, zero, None, *bad)


# ---------------------------------------------------------------- shared pivots (approximate)

def test_pivot_groups_and_zeta_against_brute_force():
    """Clustered points whose pivot cells hold several points: the oracle's group pivots (exact
    lattice positions, weights) and zeta against the numpy grouping and Legendre form."""
    rng = np.random.default_rng(5)
    centres = rng.random((6, 3)) * 60.0
    P = (centres[rng.integers(0, 6, 300)] + rng.normal(0, 2.5, (300, 3))) % 60.0
    w = rng.normal(1.0, 0.4, 300)
    for periodic in (True, False):
        r = oracle.zeta_pivots(P[:, 0], P[:, 1], P[:, 2], w, 60.0, periodic, 5, 1.0, 15.0, 4, 3.0)
        X, W, q, K = brute.pivot_groups(P[:, 0], P[:, 1], P[:, 2], w, 60.0, periodic, 15.0, 3.0)
        assert r.ngroups == len(X) < 300
        np.testing.assert_array_equal(r.gq, X)
        np.testing.assert_allclose(r.gw, W, rtol=0, atol=1e-13)
        assert abs(r.gw.sum() - w.sum()) < 1e-11
        T = brute.thresholds(5, 1.0, 15.0, 60.0, K)
        ref = brute.zeta_triangles_lattice(X, W, q, w, K, periodic, T, 5, 4)
        assert _rel(r.zeta, ref) < 1e-12


def test_pivots_with_one_point_per_group_are_exact():
    """When every pivot cell holds one point, each group pivot is that point and the approximation
    is the exact estimator (to summation order)."""
    rng = np.random.default_rng(6)
    side, h = 50.0, 2.5
    cells = rng.choice(20 ** 3, 400, replace=False)
    ijk = np.stack(np.unravel_index(cells, (20, 20, 20)), 1)
    P = (ijk + 0.1 + 0.8 * rng.random((400, 3))) * h
    w = rng.normal(1.0, 0.3, 400)
    r = oracle.zeta_pivots(P[:, 0], P[:, 1], P[:, 2], w, side, True, 6, 1.0, 12.0, 6, h * (1 + 1e-12))
    ex = oracle.zeta(P[:, 0], P[:, 1], P[:, 2], w, side, True, 6, 1.0, 12.0, 6)
    assert r.ngroups == 400
    assert r.npairs == ex.npairs
    assert _rel(r.zeta, ex.zeta) < 1e-12


def test_pivots_converge_to_exact():
    """The approximation error shrinks with the pivot cell (clustered catalogue, l_max = 4)."""
    cat = catalogs.lognormal(3000, 100.0, 3, grid=32)
    ex = oracle.zeta(cat.x, cat.y, cat.z, None, 100.0, True, 8, 4.0, 20.0, 4).zeta
    errs = []
    for h in (4.0, 2.0, 1.0, 0.5):
        r = oracle.zeta_pivots(cat.x, cat.y, cat.z, None, 100.0, True, 8, 4.0, 20.0, 4, h)
        errs.append(_rel(r.zeta, ex))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[-1] < 0.02 and errs[0] > 1e-3


def test_pivots_invalid():
    one = np.zeros(2)
    with pytest.raises(ValueError):
        oracle.zeta_pivots(one, one, one, None, 10.0, True, 2, 0.0, 2.0, 1, 0.0)
    r = oracle.zeta_pivots(np.zeros(0), np.zeros(0), np.zeros(0), None, 10.0, True, 2, 0.0, 2.0, 1, 1.0)
    assert r.ngroups == 0 and not r.zeta.any()


def test_sphere_pivots_against_brute_force_and_exact_limit():
    """Shared pivots on the sphere: against the numpy grouping and triangle form on clustered
    points; with one pixel per pivot cell (HEALPix nside 16, cells of 0.01) the exact estimator."""
    m = catalogs.sphere_cluster(300, 4, ncentre=3, spread=0.05)
    r = oracle.zeta_sphere_pivots(m.x, m.y, m.z, m.w, 5, 0.005, 0.2, 6, 0.02)
    ref, G = brute.zeta_sphere_pivots_triangles(m.x, m.y, m.z, m.w, 5, 0.005, 0.2, 6, 0.02)
    assert r.ngroups == G < 300
    assert _rel(r.zeta, ref) < 1e-12
    x, y, z = catalogs.healpix_centres(16)
    w = np.random.default_rng(1).normal(1.0, 0.5, len(x))
    rp = oracle.zeta_sphere_pivots(x, y, z, w, 4, 0.0, 0.3, 4, 0.01)
    ex = oracle.zeta_sphere(x, y, z, w, 4, 0.0, 0.3, 4)
    assert rp.ngroups == len(x) and rp.npairs == ex.npairs
    assert _rel(rp.zeta, ex.zeta) < 1e-12


def test_sphere_edge_correction_closed_forms():
    """Edge correction of the 2D multipoles: (1) N built from a known c with the closed-form
    coupling eps_m' (R_{m+m'} + R_{|m-m'|}) / 2 (R_k = 0 above m_max) is solved back; (2) R/R gives
    (1, 0, ...); (3) isotropic R gives N / R_0; (4) densities R(phi) = 1 + 0.4 cos(phi) and
    zeta(phi) = 1 + 0.3 cos(2 phi), integrated on a fine grid, give c_0 = 1, c_2 = 0.15."""
    rng = np.random.default_rng(8)
    M, nb = 5, 3
    R = np.zeros((M + 1, nb, nb))
    R[0] = 1.0 + rng.random((nb, nb))
    R[1:] = 0.3 * rng.normal(size=(M, nb, nb)) * R[0]
    c = rng.normal(size=(M + 1, nb, nb))
    N = np.zeros_like(c)
    Rk = lambda k: R[k] if k <= M else 0.0
    for m in range(M + 1):
        for mp in range(M + 1):
            N[m] += (1.0 if mp == 0 else 2.0) * 0.5 * (Rk(m + mp) + Rk(abs(m - mp))) * c[mp]
    out = oracle.edge_correct_sphere(N, R)
    assert np.abs(out - c).max() < 1e-11 * np.abs(c).max()
    rr = oracle.edge_correct_sphere(R, R)
    unit = np.zeros_like(rr)
    unit[0] = 1.0
    assert np.abs(rr - unit).max() < 1e-13
    Ri = np.zeros_like(R)
    Ri[0] = R[0]
    np.testing.assert_allclose(oracle.edge_correct_sphere(N, Ri), N / R[0], rtol=1e-13, atol=0)
    phi = np.linspace(0.0, 2 * np.pi, 4096, endpoint=False)
    dens_R = 1.0 + 0.4 * np.cos(phi)
    dens_N = (1.0 + 0.3 * np.cos(2 * phi)) * dens_R
    mom = lambda f: np.array([np.sum(f * np.cos(m * phi)) * (2 * np.pi / len(phi)) for m in range(5)])
    c2 = oracle.edge_correct_sphere(mom(dens_N)[:, None, None], mom(dens_R)[:, None, None])[:, 0, 0]
    np.testing.assert_allclose(c2, [1.0, 0.0, 0.15, 0.0, 0.0], rtol=0, atol=1e-12)


def _tridiagonal_sphere(mmax, a):
    """Coupling of the 2D edge correction for R(phi) = R_0 (1 + 2 a cos phi) / (2 pi): by
    2 cos(phi) cos(m' phi) = cos((m'+1) phi) + cos((m'-1) phi), A = I + a (sub- and super-diagonal)
    except A[0, 1] = 2 a (the m' = 1 term counts +1 and -1)."""
    A = np.eye(mmax + 1)
    for m in range(mmax):
        A[m, m + 1] += a
        A[m + 1, m] += a
    A[0, 1] = 2 * a
    return A


@pytest.mark.parametrize("mmax", [10, 16])
def test_sphere_edge_correction_high_order(mmax):
    """2D edge correction at m_max = 10 and at the oracle's cap (16), pinned without the
    coupling formula the oracle integrates: (1) R(phi) = R_0 (1 + 2 a cos phi) / (2 pi) gives the
    tridiagonal coupling of the cosine product rule, and N = R_0 A c is solved back; (2) for random
    cosine series, N(phi) = zeta(phi) R(phi) is their product taken as a discrete convolution of
    the two-sided Fourier coefficients (numpy.convolve), R_k = 0 above m_max, and c is recovered."""
    rng = np.random.default_rng(200 + mmax)
    R0, a = 1.7, 0.35
    c = rng.normal(size=mmax + 1)
    R = np.zeros((mmax + 1, 1, 1))
    R[0, 0, 0], R[1, 0, 0] = R0, a * R0
    N = (R0 * _tridiagonal_sphere(mmax, a) @ c)[:, None, None]
    assert np.abs(oracle.edge_correct_sphere(N, R)[:, 0, 0] - c).max() < 1e-12 * np.abs(c).max()
    nb = 2
    Rr = np.zeros((mmax + 1, nb, nb))
    Rr[0] = rng.uniform(1.0, 2.0, (nb, nb))
    Rr[1:] = 0.3 * rng.normal(size=(mmax, nb, nb)) * Rr[0] / np.arange(1, mmax + 1)[:, None, None]
    cr = rng.normal(size=(mmax + 1, nb, nb))
    Nr = np.zeros_like(cr)
    for i in range(nb):
        for j in range(nb):
            two = lambda v: np.concatenate([v[:0:-1], v])  # coefficients of exp(i k phi), k = -M..M
            full = np.convolve(two(cr[:, i, j]), two(Rr[:, i, j]))  # k = -2M..2M
            Nr[:, i, j] = full[2 * mmax: 3 * mmax + 1]
    assert np.abs(oracle.edge_correct_sphere(Nr, Rr) - cr).max() < 1e-11 * np.abs(cr).max()
