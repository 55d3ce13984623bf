"""Seeded synthetic workloads for the Vecchia log-likelihood.

This module is shared by the oracle tests, the GPU tests and the benchmark.
It draws inputs only: locations, the ordering, observations, covariance
parameters, and the conditioning sets (m nearest previously-ordered
neighbours).  It holds none of the log-likelihood arithmetic.  The one place
where a covariance is formed, the exact Gaussian draw of the small
configuration, uses the general Bessel form of the Matern covariance, Eq. (2),
through ``scipy.special.kv``, not the closed forms that the oracle and the
kernels use.

Shapes follow the paper's workloads: two-dimensional locations in the unit
square (Sec. V-B uses 2D fields of 180K and 260K points), random ordering
(Sec. IV-A), and conditioning-set sizes from the paper's m grid (Sec. V-D).

Draw order inside each configuration: locations, permutation, observations,
then covariance parameters.  Each configuration has a fixed seed.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_KNN_SRC = os.path.join(_HERE, "knn.c")
_KNN_LIB = os.path.join(_HERE, "libknn.so")

SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}


# --------------------------------------------------------------------------- kNN
def build_knn(force: bool = True) -> str:
    """Compile the neighbour-search library in place (gcc, OpenMP)."""
    if force or not os.path.exists(_KNN_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               "-std=c11", "-o", _KNN_LIB + ".tmp", _KNN_SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_KNN_LIB + ".tmp", _KNN_LIB)
    return _KNN_LIB


_knn = None


def _knn_lib():
    global _knn
    if _knn is None:
        if not os.path.exists(_KNN_LIB):
            build_knn()
        lib = ctypes.CDLL(_KNN_LIB)
        lib.knn_previous.restype = ctypes.c_int
        lib.knn_previous.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_int32]
        _knn = lib
    return _knn


def nearest_previous_neighbours(locs: np.ndarray, m: int, threads: int = 0) -> np.ndarray:
    """Conditioning sets J_i: for each point i the min(i, m) nearest points among 0..i-1.

    Returns an int32 array [n][m], each row sorted by (distance, index), padded with -1.
    """
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    out = np.empty((n, max(m, 0)), dtype=np.int32)
    if m == 0:
        return out
    rc = _knn_lib().knn_previous(locs.ctypes.data, n, m, out.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"knn_previous failed with code {rc}")
    return out


# --------------------------------------------------------------------- generators
def uniform_locations(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=(n, 2))


def lonlat_locations(rng: np.random.Generator, n: int, lon=(-95.0, -85.0), lat=(30.0, 40.0)) -> np.ndarray:
    """(longitude, latitude) in degrees, uniform over a lon x lat box; the default 10 x 10 degree box has
    the extent of a regional field such as the soil-moisture data of the real-data study."""
    return np.column_stack([rng.uniform(lon[0], lon[1], n), rng.uniform(lat[0], lat[1], n)])


def jittered_grid_locations(rng: np.random.Generator, n: int, jitter: float = 0.4) -> np.ndarray:
    """sqrt(n) x sqrt(n) cell centres ((i+1/2)/g, (j+1/2)/g) plus U(-jitter/g, +jitter/g) per coordinate."""
    g = math.isqrt(n)
    if g * g != n:
        raise ValueError("jittered grid needs a square n")
    c = (np.arange(g) + 0.5) / g
    xx, yy = np.meshgrid(c, c, indexing="xy")
    base = np.stack([xx.ravel(), yy.ravel()], axis=1)
    return base + rng.uniform(-jitter / g, jitter / g, size=base.shape)


def matern_bessel(d: np.ndarray, nu: float, sigma2: float, beta: float) -> np.ndarray:
    """Eq. (2) in its general Bessel form (distance scaled by beta only), C(0) = sigma2."""
    from scipy.special import gamma, kv

    d = np.asarray(d, dtype=np.float64)
    r = d / beta
    out = np.full(r.shape, sigma2, dtype=np.float64)
    pos = r > 0
    rp = r[pos]
    out[pos] = sigma2 * (2.0 ** (1.0 - nu) / gamma(nu)) * rp ** nu * kv(nu, rp)
    return out


def exact_gp_draw(rng: np.random.Generator, locs: np.ndarray, nu: float, sigma2: float, beta: float,
                  tau2: float = 0.0) -> np.ndarray:
    """z = L eps with L the dense Cholesky factor of the covariance of the ordered locations."""
    diff = locs[:, None, :] - locs[None, :, :]
    d = np.sqrt((diff ** 2).sum(-1))
    cov = matern_bessel(d, nu, sigma2, beta) + tau2 * np.eye(len(locs))
    L = np.linalg.cholesky(cov)
    return L @ rng.standard_normal(len(locs))


# ------------------------------------------------------------------- workloads
@dataclass
class Field:
    """One spatial field, already in the ordering tau."""
    locs: np.ndarray          # [n][2] float64
    z: np.ndarray             # [n] float64
    nbr: np.ndarray           # [n][m] int32, -1 padded
    m: int
    nu: float
    thetas: np.ndarray        # [P][3] float64: (sigma2, beta, tau2) per parameter vector

    @property
    def n(self) -> int:
        return int(self.locs.shape[0])


@dataclass
class Workload:
    name: str
    fields: list = field(default_factory=list)
    with_grad: bool = False
    description: str = ""


def _ordered(rng, locs):
    perm = rng.permutation(len(locs))
    return np.ascontiguousarray(locs[perm])


def config_small(n: int = 2000, m: int = 30, seed: int = SEEDS[1], knn_threads: int = 0) -> Workload:
    """n=2,000 uniform points, random order, m=30, nu=0.5, theta=(1, 0.1, 0); z an exact GP draw."""
    rng = np.random.default_rng(seed)
    locs = _ordered(rng, uniform_locations(rng, n))
    theta = np.array([[1.0, 0.1, 0.0]])
    z = exact_gp_draw(rng, locs, 0.5, 1.0, 0.1, 0.0)
    nbr = nearest_previous_neighbours(locs, m, knn_threads)
    return Workload("n2k_m30_nu0.5", [Field(locs, z, nbr, m, 0.5, theta)], False,
                    "n=2000 uniform, m=30, Matern nu=0.5, exact GP draw, forward only")


def config_grid(n: int = 250_000, m: int = 60, seed: int = SEEDS[2], knn_threads: int = 0) -> Workload:
    """n=250,000 jittered grid, random order, m=60, nu=1.5, theta=(1, 0.05, 1e-6), z iid N(0,1)."""
    rng = np.random.default_rng(seed)
    locs = _ordered(rng, jittered_grid_locations(rng, n))
    z = rng.standard_normal(n)
    theta = np.array([[1.0, 0.05, 1e-6]])
    nbr = nearest_previous_neighbours(locs, m, knn_threads)
    return Workload("n250k_m60_nu1.5_grid", [Field(locs, z, nbr, m, 1.5, theta)], False,
                    "n=250000 jittered grid, m=60, Matern nu=1.5, forward only")


def config_large(n: int = 1_000_000, m: int = 120, seed: int = SEEDS[3], knn_threads: int = 0) -> Workload:
    """n=1,000,000 uniform, random order, m=120, nu=0.5, theta=(1.5, 0.03, 1e-4), z iid; value + gradient."""
    rng = np.random.default_rng(seed)
    locs = _ordered(rng, uniform_locations(rng, n))
    z = rng.standard_normal(n)
    theta = np.array([[1.5, 0.03, 1e-4]])
    nbr = nearest_previous_neighbours(locs, m, knn_threads)
    return Workload("n1M_m120_nu0.5", [Field(locs, z, nbr, m, 0.5, theta)], True,
                    "n=1000000 uniform, m=120, Matern nu=0.5, value + gradient")


def config_multitheta(n: int = 200_000, m: int = 60, ntheta: int = 64, seed: int = SEEDS[4],
                      knn_threads: int = 0) -> Workload:
    """n=200,000 uniform, m=60, nu=2.5, 64 parameter vectors; value + gradient for each."""
    rng = np.random.default_rng(seed)
    locs = _ordered(rng, uniform_locations(rng, n))
    z = rng.standard_normal(n)
    thetas = np.stack([rng.uniform(0.5, 2.0, ntheta), rng.uniform(0.01, 0.3, ntheta),
                       rng.uniform(0.0, 1e-3, ntheta)], axis=1)
    nbr = nearest_previous_neighbours(locs, m, knn_threads)
    return Workload(f"n200k_m60_nu2.5_{ntheta}theta", [Field(locs, z, nbr, m, 2.5, thetas)], True,
                    f"n=200000 uniform, m=60, Matern nu=2.5, {ntheta} parameter vectors, value + gradient")


def config_multifield(nfields: int = 32, seed: int = SEEDS[5], n_lo: float = 1e4, n_hi: float = 5e5,
                      m_lo: int = 10, m_hi: int = 150, knn_threads: int = 0) -> Workload:
    """32 fields, n log-uniform on [1e4, 5e5], m uniform on {10..150}, nu=1.5, per-field theta."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), nfields))).astype(np.int64)
    ms = rng.integers(m_lo, m_hi + 1, nfields)
    th = np.stack([rng.uniform(0.5, 2.0, nfields), rng.uniform(0.02, 0.2, nfields),
                   rng.uniform(0.0, 1e-3, nfields)], axis=1)
    fields = []
    for f in range(nfields):
        locs = _ordered(rng, uniform_locations(rng, int(ns[f])))
        z = rng.standard_normal(int(ns[f]))
        nbr = nearest_previous_neighbours(locs, int(ms[f]), knn_threads)
        fields.append(Field(locs, z, nbr, int(ms[f]), 1.5, th[f:f + 1].copy()))
    return Workload(f"{nfields}fields_nu1.5", fields, True,
                    f"{nfields} fields, n log-uniform [1e4,5e5], m uniform 10..150, Matern nu=1.5, value + gradient")


def small_field(rng: np.random.Generator, n: int, m: int, nu: float, theta, grid: bool = False) -> Field:
    """A small random field for parity tests (uniform or jittered-grid points, z iid N(0,1))."""
    locs = jittered_grid_locations(rng, n) if grid else uniform_locations(rng, n)
    locs = _ordered(rng, locs)
    z = rng.standard_normal(n)
    nbr = nearest_previous_neighbours(locs, m)
    return Field(locs, z, nbr, m, nu, np.atleast_2d(np.asarray(theta, dtype=np.float64)))
