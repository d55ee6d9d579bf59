"""Seeded synthetic catalogues shared by the oracle tests, the GPU tests and the benchmark.

This module only draws inputs: positions in a cube and weights. It contains none of the
estimator's arithmetic (no binning, no harmonics, no lattice), so the oracle and the HIP
path can both take their inputs from here without sharing any part of the method.

Workloads (all positions in FP64, box side ``box``):

* ``uniform``     -- i.i.d. uniform points in [0, box)^3.
* ``lognormal``   -- points Poisson-sampled (conditioned on the total N) from a log-normal
  density field: a Gaussian random field with power-law spectrum P(k) ~ k^slope on a
  ``grid``^3 mesh, rescaled to standard deviation ``sigma`` and exponentiated.
* ``gaussian_weights`` -- w = mean + sd * N(0, 1) from an independent stream.
* ``mock_sizes``  -- catalogue sizes drawn log-uniform in [lo, hi].
* ``data_minus_randoms`` -- clustered data plus uniform randoms in a non-periodic cube, the
  randoms weighted -N_d/N_r so that the combined field has zero mean.
* ``healpix_centres`` -- unit vectors of the pixel centres of a HEALPix map (RING scheme,
  Gorski et al. 2005): the pixel layout of the maps the paper measures on.
* ``sphere_field``    -- a log-normal density contrast (rho - 1) sampled at points on the unit
  sphere from a 3D log-normal field (trilinear interpolation), as map values (convergence-like:
  zero mean, skewed).
* ``sphere_map``      -- ``healpix_centres`` with ``sphere_field`` values: a full-sky map.
* ``sphere_cluster``  -- clustered points on the sphere (Gaussian caps around random centres,
  the poles included), for small-size parity cases.
* ``radec_to_unit``   -- (ra, dec) in radians to unit vectors.

The paper measures on HEALPix maps and N-body simulation products that are not available
here; these generators stand in for them with the shapes, sizes and clustering of the
three-point workloads the estimator is meant for.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform",
    "lognormal_field",
    "lognormal",
    "gaussian_weights",
    "mock_sizes",
    "data_minus_randoms",
    "Catalog",
    "radec_to_unit",
    "healpix_centres",
    "sphere_field",
    "sphere_field_sampler",
    "sphere_map",
    "sphere_cluster",
    "SphereMap",
]


class Catalog:
    """Plain container: x, y, z, w (float64 arrays), box side and periodic flag."""

    def __init__(self, x, y, z, w, box, periodic, name=""):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.box = float(box)
        self.periodic = bool(periodic)
        self.name = name

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "Catalog":
        idx = np.asarray(idx)
        return Catalog(self.x[idx], self.y[idx], self.z[idx], self.w[idx], self.box,
                       self.periodic, self.name + "[subset]")


def uniform(n: int, box: float, seed: int) -> Catalog:
    """n uniform points in [0, box)^3 from numpy's PCG64 stream ``seed``; unit weights."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * box
    # random() is in [0,1); multiplying by box can round up to box itself in rare cases.
    pos = np.minimum(pos, np.nextafter(box, 0.0))
    return Catalog(pos[:, 0], pos[:, 1], pos[:, 2], np.ones(n), box, True, f"uniform(n={n},seed={seed})")


def lognormal_field(grid: int, box: float, seed: int, slope: float = -1.5,
                    sigma: float = 1.0) -> np.ndarray:
    """Normalised log-normal density rho (mean 1) on a grid^3 mesh.

    Steps: white noise N(0,1) on the mesh -> rfftn -> multiply by sqrt(P(k)) with
    P(k) = k^slope (P(0) = 0) -> irfftn -> G; G is shifted to zero mean and scaled to
    standard deviation ``sigma``; rho = exp(G) / mean(exp(G)).
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((grid, grid, grid))
    fk = np.fft.rfftn(white)
    del white
    kx = 2.0 * np.pi * np.fft.fftfreq(grid, d=box / grid)
    kz = 2.0 * np.pi * np.fft.rfftfreq(grid, d=box / grid)
    k2 = (kx[:, None, None] ** 2 + kx[None, :, None] ** 2) + kz[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)  # sqrt(k^slope) = (k^2)^(slope/4)
    fk *= amp
    del amp, k2
    g = np.fft.irfftn(fk, s=(grid, grid, grid), axes=(0, 1, 2))
    del fk
    g -= g.mean()
    g *= sigma / g.std()
    rho = np.exp(g)
    rho /= rho.mean()
    return rho


def _sample_from_field(rho: np.ndarray, n: int, box: float, rng) -> np.ndarray:
    """Draw exactly n points with cell probabilities proportional to rho, uniform in-cell."""
    grid = rho.shape[0]
    cdf = np.cumsum(rho.ravel(), dtype=np.float64)
    cdf /= cdf[-1]
    u = rng.random(n)
    cell = np.searchsorted(cdf, u, side="right")
    cell = np.minimum(cell, grid ** 3 - 1)
    ix, rem = np.divmod(cell, grid * grid)
    iy, iz = np.divmod(rem, grid)
    h = box / grid
    off = rng.random((n, 3))
    pos = np.empty((n, 3))
    pos[:, 0] = (ix + off[:, 0]) * h
    pos[:, 1] = (iy + off[:, 1]) * h
    pos[:, 2] = (iz + off[:, 2]) * h
    return np.minimum(pos, np.nextafter(box, 0.0))


def lognormal(n: int, box: float, seed: int, grid: int = 256, slope: float = -1.5,
              sigma: float = 1.0, periodic: bool = True) -> Catalog:
    """n points Poisson-sampled (conditioned on n) from a log-normal field; unit weights.

    The field and the positions use one PCG64 stream ``seed`` (field first, then positions).
    """
    rng = np.random.default_rng(seed)
    field_seed = int(rng.integers(0, 2**63 - 1))
    rho = lognormal_field(grid, box, field_seed, slope, sigma)
    pos = _sample_from_field(rho, n, box, rng)
    return Catalog(pos[:, 0], pos[:, 1], pos[:, 2], np.ones(n), box, periodic,
                   f"lognormal(n={n},box={box},seed={seed},grid={grid})")


def gaussian_weights(n: int, seed: int, mean: float = 1.0, sd: float = 0.1) -> np.ndarray:
    """w = mean + sd * N(0,1) from an independent PCG64 stream ``seed``."""
    rng = np.random.default_rng(seed)
    return mean + sd * rng.standard_normal(n)


def mock_sizes(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """``count`` catalogue sizes, round(exp(U(ln lo, ln hi)))."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def data_minus_randoms(n_data: int, n_rand: int, box: float, seed_data: int, seed_rand: int,
                       grid: int = 256) -> Catalog:
    """Clustered data (w = 1) plus uniform randoms (w = -n_data/n_rand), non-periodic cube."""
    d = lognormal(n_data, box, seed_data, grid=grid, periodic=False)
    r = uniform(n_rand, box, seed_rand)
    x = np.concatenate([d.x, r.x])
    y = np.concatenate([d.y, r.y])
    z = np.concatenate([d.z, r.z])
    w = np.concatenate([np.ones(n_data), np.full(n_rand, -n_data / n_rand)])
    return Catalog(x, y, z, w, box, False,
                   f"data_minus_randoms(nd={n_data},nr={n_rand},box={box})")


# ---------------------------------------------------------------- the unit sphere

class SphereMap:
    """Plain container of a field on the unit sphere: unit vectors x, y, z and values w."""

    def __init__(self, x, y, z, w, name=""):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.name = name

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def radec_to_unit(ra, dec):
    """(cos dec cos ra, cos dec sin ra, sin dec) as three float64 arrays."""
    ra = np.asarray(ra, dtype=np.float64)
    dec = np.asarray(dec, dtype=np.float64)
    c = np.cos(dec)
    return (np.ascontiguousarray(c * np.cos(ra)), np.ascontiguousarray(c * np.sin(ra)),
            np.ascontiguousarray(np.sin(dec)))


def healpix_centres(nside: int):
    """Unit vectors of the 12 nside^2 pixel centres of a HEALPix map, RING order.

    Rings i = 1..4 nside - 1 from the north pole. Polar caps (i < nside, and the mirror rings
    i > 3 nside): z = +-(1 - k^2 / (3 nside^2)) with k = i or 4 nside - i, 4k pixels at
    phi = (pi / (2k)) (j - 1/2). Equatorial belt (nside <= i <= 3 nside): z = 4/3 - 2i / (3 nside),
    4 nside pixels at phi = (pi / (2 nside)) (j - s/2), s = (i - nside + 1) mod 2, j = 1..4 nside.
    """
    ns = int(nside)
    npix = 12 * ns * ns
    out = [np.empty(npix) for _ in range(3)]
    at = 0
    # ring by ring into preallocated outputs: the peak memory stays at the three outputs
    for i in range(1, 4 * ns):
        if i < ns or i > 3 * ns:
            k = i if i < ns else 4 * ns - i
            z = 1.0 - k * k / (3.0 * ns * ns)
            if i > 3 * ns:
                z = -z
            j = np.arange(1, 4 * k + 1, dtype=np.float64)
            phi = (np.pi / (2.0 * k)) * (j - 0.5)
        else:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            sft = (i - ns + 1) % 2
            j = np.arange(1, 4 * ns + 1, dtype=np.float64)
            phi = (np.pi / (2.0 * ns)) * (j - 0.5 * sft)
        zr = np.full(phi.shape, z)
        st = np.sqrt(np.maximum(0.0, (1.0 - zr) * (1.0 + zr)))
        x, y = st * np.cos(phi), st * np.sin(phi)
        # unit length to rounding: renormalise so |v|^2 = 1 within a few ulp
        r = np.sqrt(x * x + y * y + zr * zr)
        m = len(phi)
        out[0][at:at + m] = x / r
        out[1][at:at + m] = y / r
        out[2][at:at + m] = zr / r
        at += m
    assert at == npix
    return tuple(out)


def sphere_field_sampler(seed: int, grid: int = 256, slope: float = -1.5, sigma: float = 0.5):
    """The sampling function behind ``sphere_field``: builds the 3D field once and returns
    f(x, y, z) -> rho - 1 at those unit vectors (for maps generated in slices)."""
    side = 2.5
    rho = lognormal_field(grid, side, seed, slope, sigma)
    return lambda x, y, z: _trilinear(rho, side, x, y, z)


def sphere_field(x, y, z, seed: int, grid: int = 256, slope: float = -1.5, sigma: float = 0.5) -> np.ndarray:
    """rho - 1 of a log-normal field (``lognormal_field`` on a periodic grid^3 mesh of side 2.5
    centred on the origin) at the unit vectors (x, y, z), trilinear interpolation."""
    return sphere_field_sampler(seed, grid, slope, sigma)(x, y, z)


def _trilinear(rho, side, x, y, z):
    grid = rho.shape[0]
    h = side / grid
    out = np.empty(len(x))
    step = 1 << 22
    for a in range(0, len(x), step):
        b = min(len(x), a + step)
        u = np.stack([x[a:b], y[a:b], z[a:b]], 1) * (1.0 / h) + (0.5 * side / h - 0.5)
        i0 = np.floor(u).astype(np.int64)
        f = u - i0
        i0 %= grid
        i1 = (i0 + 1) % grid
        acc = np.zeros(b - a)
        for cx in (0, 1):
            ix = i1[:, 0] if cx else i0[:, 0]
            wx = f[:, 0] if cx else 1.0 - f[:, 0]
            for cy in (0, 1):
                iy = i1[:, 1] if cy else i0[:, 1]
                wy = f[:, 1] if cy else 1.0 - f[:, 1]
                for cz in (0, 1):
                    iz = i1[:, 2] if cz else i0[:, 2]
                    wz = f[:, 2] if cz else 1.0 - f[:, 2]
                    acc += wx * wy * wz * rho[ix, iy, iz]
        out[a:b] = acc - 1.0
    return out


def sphere_map(nside: int, seed: int, grid: int = 256, sigma: float = 0.5) -> SphereMap:
    """A full-sky HEALPix map (``healpix_centres``) with ``sphere_field`` values."""
    x, y, z = healpix_centres(nside)
    w = sphere_field(x, y, z, seed, grid=grid, sigma=sigma)
    return SphereMap(x, y, z, w, f"healpix(nside={nside},seed={seed})")


def sphere_cluster(n: int, seed: int, ncentre: int = 8, spread: float = 0.1) -> SphereMap:
    """n points in Gaussian caps (angular sd ``spread``) around ``ncentre`` random centres, the
    two poles among them, and the exact north pole as the last point; weights N(1, 0.5^2)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(ncentre, 3))
    c[0] = (0.0, 0.0, 1.0)
    c[1 % ncentre] = (0.0, 0.0, -1.0) if ncentre > 1 else c[1 % ncentre]
    c /= np.linalg.norm(c, axis=1)[:, None]
    k = rng.integers(0, ncentre, n - 1)
    v = c[k] + spread * rng.normal(size=(n - 1, 3))
    v = np.concatenate([v, [[0.0, 0.0, 1.0]]])
    v /= np.linalg.norm(v, axis=1)[:, None]
    w = rng.normal(1.0, 0.5, n)
    return SphereMap(v[:, 0], v[:, 1], v[:, 2], w, f"sphere_cluster(n={n},seed={seed})")

