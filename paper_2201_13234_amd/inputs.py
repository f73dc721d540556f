"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module only draws random inputs; it contains none of the diagram's
arithmetic.  The paper evaluates uniformly random ("Poisson") sites on
regular grids (arXiv 2201.13234, Sec. 3 problem statement and Sec. 4); the
generators below stand in for those workloads.  Every array is drawn with
numpy's PCG64 generator from an explicit seed, so the device library and the
oracle receive bit-identical inputs.

Conventions: L_a = n_a (unit voxels), coordinates uniform in [0, L_a) with a
value that rounds up to L_a clamped to the largest double below L_a.
"""
from dataclasses import dataclass, field
import math

import numpy as np

VORONOI, LAGUERRE, JOHNSON_MEHL = 0, 1, 2
KIND_NAMES = {VORONOI: "voronoi", LAGUERRE: "laguerre", JOHNSON_MEHL: "johnson_mehl"}


@dataclass
class Workload:
    name: str
    n: tuple            # voxels per axis, axis 0 fastest
    L: tuple            # domain lengths
    kind: int
    periodic: bool
    coords: np.ndarray  # [nsites, ndim] float64
    param: np.ndarray = None  # [nsites] float64 (w_s or t_s) or None
    growth: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def nsites(self):
        return int(self.coords.shape[0])

    @property
    def nvox(self):
        return int(np.prod(self.n))

    @property
    def shape(self):
        """numpy shape of the label image (slowest axis first)."""
        return tuple(reversed(self.n))


def uniform_sites(rng, nsites, L):
    L = np.asarray(L, dtype=np.float64)
    u = rng.random((int(nsites), L.shape[0])) * L
    top = np.nextafter(L, 0.0)
    return np.minimum(u, top)


def clustered_sites(rng, nsites, L, nclusters, sigma, periodic=True):
    """Sites in Gaussian clusters: centres uniform in the box, each site a
    centre plus N(0, sigma^2) per axis, wrapped into [0, L) (periodic) or
    redrawn uniformly when it falls outside (non-periodic)."""
    L = np.asarray(L, dtype=np.float64)
    centres = rng.random((int(nclusters), L.shape[0])) * L
    pick = rng.integers(0, int(nclusters), int(nsites))
    c = centres[pick] + sigma * rng.standard_normal((int(nsites), L.shape[0]))
    if periodic:
        c = np.mod(c, L)
    else:
        out = (c < 0.0) | (c >= L)
        c = np.where(out, rng.random(c.shape) * L, c)
    return np.minimum(c, np.nextafter(L, 0.0))


def spacing(n_vox, nsites, ndim):
    """Mean site spacing (V / N_s)^(1/d) for unit voxels."""
    return (float(n_vox) / float(nsites)) ** (1.0 / ndim)


def lognormal_weights(rng, nsites, median_radius, sigma=0.3):
    """Laguerre weights w = r^2 with r = median * exp(sigma * Z)."""
    r = median_radius * np.exp(sigma * rng.standard_normal(int(nsites)))
    return r * r


def make(n, kind, periodic, nsites, seed, tmax=None, growth=1.0, sigma=0.3,
         name=None):
    """One workload: uniform sites, then the kind's parameter."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in n)
    rng = np.random.default_rng(seed)
    coords = uniform_sites(rng, nsites, L)
    sp = spacing(np.prod(n), nsites, len(n))
    param = None
    if kind == LAGUERRE:
        param = lognormal_weights(rng, nsites, 0.5 * sp, sigma)
    elif kind == JOHNSON_MEHL:
        if tmax is None:
            tmax = 1.92 * sp
        param = rng.uniform(0.0, tmax, int(nsites))
    return Workload(name=name or f"{KIND_NAMES[kind]}_{'x'.join(map(str, n))}_{nsites}",
                    n=n, L=L, kind=kind, periodic=bool(periodic), coords=coords,
                    param=param, growth=float(growth),
                    meta=dict(seed=seed, spacing=sp))


# The five configurations of the benchmark plan.
def m1():
    """3D Voronoi 64^3, 256 sites, periodic, seed 1."""
    return make((64, 64, 64), VORONOI, True, 256, 1, name="M1_voronoi_64^3_256")


def m2():
    """3D Voronoi 512^3, 100,000 sites, periodic, seed 2."""
    return make((512, 512, 512), VORONOI, True, 100_000, 2, name="M2_voronoi_512^3_100k")


def m3():
    """3D Laguerre 512^3, 20,000 sites, non-periodic, w = r^2, r lognormal
    (median half the mean spacing, sigma 0.3), seed 3."""
    return make((512, 512, 512), LAGUERRE, False, 20_000, 3, name="M3_laguerre_512^3_20k")


def m4():
    """3D Johnson-Mehl 384^3, 50,000 sites, periodic, t ~ U[0,20], v = 1, seed 4."""
    return make((384, 384, 384), JOHNSON_MEHL, True, 50_000, 4, tmax=20.0,
                name="M4_jm_384^3_50k")


CONFIGS = {"M1": m1, "M2": m2, "M3": m3, "M4": m4}


def clustered(seed, n=(256, 256, 256), nsites=40_000, nclusters=200, sigma=6.0):
    """Non-uniform class for the autotuner: 3D Voronoi, periodic, sites in
    Gaussian clusters (default 200 clusters of sigma 6 voxels on 256^3)."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in n)
    rng = np.random.default_rng(seed)
    coords = clustered_sites(rng, nsites, L, nclusters, sigma, periodic=True)
    return Workload(name=f"clustered_voronoi_{'x'.join(map(str, n))}_{nsites}_seed{seed}", n=n, L=L,
                    kind=VORONOI, periodic=True, coords=coords, meta=dict(seed=seed, nclusters=nclusters,
                                                                          sigma=sigma))


def stream_job(j, side_scale=1.0):
    """Job j of the request stream (seed 10000 + j): 30% 2D with sides
    U{256..4096}, 70% 3D with sides U{64..512} (per axis), N_s U{10..20000},
    kind uniform, boundary Bernoulli(1/2).  side_scale shrinks the sides for
    short runs (1.0 = the full stream)."""
    rng = np.random.default_rng(10_000 + j)
    if rng.random() < 0.3:
        n = tuple(int(rng.integers(256, 4097)) for _ in range(2))
    else:
        n = tuple(int(rng.integers(64, 513)) for _ in range(3))
    if side_scale != 1.0:
        n = tuple(max(8, int(round(v * side_scale))) for v in n)
    nsites = int(rng.integers(10, 20_001))
    kind = int(rng.integers(0, 3))
    periodic = bool(rng.integers(0, 2))
    seed = int(rng.integers(0, 2**62))
    return make(n, kind, periodic, nsites, seed, name=f"job{j}")


def arrivals(n_jobs, rate, seed=99):
    """Poisson arrival times (exponential gaps at the given rate, per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, int(n_jobs)))
