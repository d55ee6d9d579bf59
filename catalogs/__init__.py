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
