"""ORACLE — TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU reference for the Vecchia log-likelihood and its gradient
(Eq. (7) evaluated as in Algorithm 1 of Pan et al.; the gradient is the
derivative of each conditional term).  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library.  The arithmetic lives in ``vecchia_oracle.c``; this
file only builds it and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vecchia_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle library in place with gcc."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_terms.restype = ctypes.c_int64
        lib.oracle_terms.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P, P,
                                     ctypes.c_int64, P, P, ctypes.c_int32]
        lib.oracle_loglik.restype = ctypes.c_int64
        lib.oracle_loglik.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P, P, P,
                                      ctypes.c_int32]
        lib.oracle_matern.restype = None
        lib.oracle_matern.argtypes = [P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P]
        lib.oracle_sum.restype = ctypes.c_double
        lib.oracle_sum.argtypes = [P, ctypes.c_int64]
        lib.oracle_knn_rows.restype = ctypes.c_int64
        lib.oracle_knn_rows.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int32]
        lib.oracle_exact_loglik.restype = ctypes.c_int64
        lib.oracle_exact_loglik.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P, P]
        lib.oracle_morton_order.restype = ctypes.c_int64
        lib.oracle_morton_order.argtypes = [P, ctypes.c_int64, P]
        I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.oracle_terms_cov.restype = I64
        lib.oracle_terms_cov.argtypes = [P, P, P, I64, I32, I32, I32, D, P, P, I64, P, P, I32]
        lib.oracle_loglik_cov.restype = I64
        lib.oracle_loglik_cov.argtypes = [P, P, P, I64, I32, I32, I32, D, P, P, P, I32]
        lib.oracle_cov_values.restype = I64
        lib.oracle_cov_values.argtypes = [P, I64, I32, I32, D, D, D, P, P]
        lib.oracle_distances.restype = I64
        lib.oracle_distances.argtypes = [P, P, I64, I32, P]
        lib.oracle_knn_rows_metric.restype = I64
        lib.oracle_knn_rows_metric.argtypes = [P, I64, I32, I32, P, I64, P, I32]
        lib.oracle_knn_query.restype = I64
        lib.oracle_knn_query.argtypes = [P, I64, P, I64, I32, I32, P, I32]
        lib.oracle_maxmin_order.restype = I64
        lib.oracle_maxmin_order.argtypes = [P, I64, ctypes.c_uint64, P]
        lib.oracle_random_order.restype = I64
        lib.oracle_random_order.argtypes = [I64, ctypes.c_uint64, P]
        lib.oracle_mix64.restype = ctypes.c_uint64
        lib.oracle_mix64.argtypes = [ctypes.c_uint64]
        lib.oracle_predict.restype = I64
        lib.oracle_predict.argtypes = [P, P, I64, P, I64, P, I32, I32, I32, D, P, P, P, I32]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    """Bad arguments (code < 0) or a failed conditional (code = i + 1 of the first failure)."""

    def __init__(self, code: int):
        self.code = int(code)
        what = "invalid argument" if code == -1 else "out of memory" if code == -2 else \
            f"non-positive pivot or conditional variance at point {code - 1}"
        super().__init__(f"oracle: {what}")


def _prep(locs, z, nbr, m):
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = locs.shape[0]
    if locs.shape != (n, 2) or z.shape != (n,):
        raise ValueError("locs must be [n][2] and z [n]")
    if m > 0:
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        if nbr.shape != (n, m):
            raise ValueError("nbr must be [n][m]")
    else:
        nbr = np.zeros((max(n, 1), 1), dtype=np.int32)
    return locs, z, nbr, n


# covariance models: family (Matern, Eq. (2); power exponential, Sec. V-C) and
# metric (Euclidean on (x, y); great-circle on (longitude, latitude) degrees, km)
MATERN, POWEXP = 0, 1
EUCLIDEAN, GREAT_CIRCLE = 0, 1
EARTH_RADIUS_KM = 6371.0


def _cov(cov):
    family, metric, smooth = cov
    return int(family), int(metric), float(smooth)


def terms_cov(locs, z, nbr, m: int, cov, theta, idx=None, with_grad: bool = False, threads: int = 0,
              raise_on_fail: bool = True):
    """Per-conditional l_i (and gradient) under a covariance model cov = (family, metric, smoothness)."""
    locs, z, nbr, n = _prep(locs, z, nbr, m)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    if idx is None:
        nidx = n
        idx_p = None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nidx = idx.shape[0]
        idx_p = idx.ctypes.data
    ell = np.empty(max(nidx, 1), dtype=np.float64)
    g = np.empty((max(nidx, 1), 3), dtype=np.float64) if with_grad else None
    rc = _load().oracle_terms_cov(locs.ctypes.data, z.ctypes.data, nbr.ctypes.data, n, m, *_cov(cov),
                                  th.ctypes.data, idx_p, nidx, ell.ctypes.data,
                                  g.ctypes.data if g is not None else None, threads)
    if rc < 0 or (rc > 0 and raise_on_fail):
        raise OracleError(rc)
    ell = ell[:nidx]
    return (ell, g[:nidx]) if with_grad else ell


def loglik_cov(locs, z, nbr, m: int, cov, theta, with_grad: bool = False, threads: int = 0):
    """Vecchia log-likelihood (and gradient) under a covariance model cov = (family, metric, smoothness)."""
    locs, z, nbr, n = _prep(locs, z, nbr, m)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    out = np.zeros(1)
    g = np.zeros(3) if with_grad else None
    rc = _load().oracle_loglik_cov(locs.ctypes.data, z.ctypes.data, nbr.ctypes.data, n, m, *_cov(cov),
                                   th.ctypes.data, out.ctypes.data, g.ctypes.data if g is not None else None,
                                   threads)
    if rc != 0:
        raise OracleError(rc)
    return (float(out[0]), g) if with_grad else float(out[0])


def cov_values(d, cov, sigma2: float, beta: float, with_dbeta: bool = False):
    """The oracle's covariance values (and d/dbeta) of a model at distances d."""
    d = np.ascontiguousarray(d, dtype=np.float64).ravel()
    out = np.empty_like(d)
    db = np.empty_like(d) if with_dbeta else None
    rc = _load().oracle_cov_values(d.ctypes.data, d.size, *_cov(cov), float(sigma2), float(beta), out.ctypes.data,
                                   db.ctypes.data if db is not None else None)
    if rc != 0:
        raise OracleError(rc)
    return (out, db) if with_dbeta else out


def distances(a, b, metric: int):
    """Distances between matching rows of a and b ([n][2]): Euclidean, or great-circle km on (lon, lat) degrees."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 2)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1, 2)
    out = np.empty(max(a.shape[0], 1))
    rc = _load().oracle_distances(a.ctypes.data, b.ctypes.data, a.shape[0], int(metric), out.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return out[:a.shape[0]]


def knn_query(ref, q, m: int, metric: int = EUCLIDEAN, threads: int = 0):
    """Neighbour sets of prediction points: the min(n_ref, m) nearest reference points of each query
    by (key, index), -1 padded; [nq][m] int32."""
    ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(-1, 2)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 2)
    out = np.empty((max(q.shape[0], 1), max(m, 1)), dtype=np.int32)
    rc = _load().oracle_knn_query(ref.ctypes.data, ref.shape[0], q.ctypes.data, q.shape[0], int(m), int(metric),
                                  out.ctypes.data, int(threads))
    if rc != 0:
        raise OracleError(rc)
    return out[:q.shape[0], :m]


def predict(ref, zref, q, nbr, m: int, cov, theta, threads: int = 0, raise_on_fail: bool = True):
    """Vecchia kriging: conditional mean and variance (of a new observation) at each prediction point."""
    ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(-1, 2)
    zref = np.ascontiguousarray(zref, dtype=np.float64).ravel()
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 2)
    nq = q.shape[0]
    nbr = np.ascontiguousarray(nbr, dtype=np.int32).reshape(nq, m) if m > 0 else np.zeros((max(nq, 1), 1),
                                                                                           dtype=np.int32)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    mean = np.empty(max(nq, 1))
    var = np.empty(max(nq, 1))
    rc = _load().oracle_predict(ref.ctypes.data, zref.ctypes.data, ref.shape[0], q.ctypes.data, nq, nbr.ctypes.data,
                                int(m), *_cov(cov), th.ctypes.data, mean.ctypes.data, var.ctypes.data, int(threads))
    if rc < 0 or (rc > 0 and raise_on_fail):
        raise OracleError(rc)
    return mean[:nq], var[:nq]


def terms(locs, z, nbr, m: int, nu: float, theta, idx=None, with_grad: bool = False, threads: int = 0,
          raise_on_fail: bool = True):
    """Per-conditional l_i (and dl_i/d(sigma2, beta, tau2)) for the points idx (default all)."""
    locs, z, nbr, n = _prep(locs, z, nbr, m)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    if idx is None:
        nidx = n
        idx_p = None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nidx = idx.shape[0]
        idx_p = idx.ctypes.data
    ell = np.empty(max(nidx, 1), dtype=np.float64)
    g = np.empty((max(nidx, 1), 3), dtype=np.float64) if with_grad else None
    rc = _load().oracle_terms(locs.ctypes.data, z.ctypes.data, nbr.ctypes.data, n, m, float(nu), th.ctypes.data,
                              idx_p, nidx, ell.ctypes.data, g.ctypes.data if g is not None else None, threads)
    if rc < 0 or (rc > 0 and raise_on_fail):
        raise OracleError(rc)
    ell = ell[:nidx]
    return (ell, g[:nidx]) if with_grad else ell


def loglik(locs, z, nbr, m: int, nu: float, theta, with_grad: bool = False, threads: int = 0):
    """Sum of l_i (Neumaier, ascending i); with_grad also returns the gradient (sigma2, beta, tau2)."""
    locs, z, nbr, n = _prep(locs, z, nbr, m)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    out = np.zeros(1)
    g = np.zeros(3) if with_grad else None
    rc = _load().oracle_loglik(locs.ctypes.data, z.ctypes.data, nbr.ctypes.data, n, m, float(nu), th.ctypes.data,
                               out.ctypes.data, g.ctypes.data if g is not None else None, threads)
    if rc != 0:
        raise OracleError(rc)
    return (float(out[0]), g) if with_grad else float(out[0])


def matern(d, nu: float, sigma2: float, beta: float, with_dbeta: bool = False):
    """The oracle's covariance values (and d/dbeta) at distances d."""
    d = np.ascontiguousarray(d, dtype=np.float64).ravel()
    out = np.empty_like(d)
    db = np.empty_like(d) if with_dbeta else None
    _load().oracle_matern(d.ctypes.data, d.size, float(nu), float(sigma2), float(beta), out.ctypes.data,
                          db.ctypes.data if db is not None else None)
    return (out, db) if with_dbeta else out


def compensated_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return float(_load().oracle_sum(x.ctypes.data, x.size))


def knn_rows(locs, m: int, rows=None, threads: int = 0, metric: int = EUCLIDEAN):
    """Conditioning sets by brute force: for each row i, the min(i, m) nearest j < i by (key, index), -1
    padded, the key being the squared distance (Euclidean) or the haversine value (great-circle); returns
    [len(rows)][m] int32 (all rows by default)."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    if locs.shape != (n, 2):
        raise ValueError("locs must be [n][2]")
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((max(rows.size, 1), max(m, 1)), dtype=np.int32)
    rc = _load().oracle_knn_rows_metric(locs.ctypes.data, n, int(m), int(metric), rows.ctypes.data, rows.size,
                                        out.ctypes.data, int(threads))
    if rc != 0:
        raise OracleError(rc)
    return out[:rows.size, :m]


def morton_order(locs):
    """Point indices in Morton (Z-order) order over the bounding box, ties by index."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    perm = np.empty(max(n, 1), dtype=np.int64)
    rc = _load().oracle_morton_order(locs.ctypes.data, n, perm.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return perm[:n]


def maxmin_order(locs, seed: int = 0):
    """Approximate maxmin ordering (rounds of per-cell elections over finer and finer grids, each round in
    hashed-index order); returns the permutation."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    perm = np.empty(max(n, 1), dtype=np.int64)
    rc = _load().oracle_maxmin_order(locs.ctypes.data, n, ctypes.c_uint64(seed & (2 ** 64 - 1)), perm.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return perm[:n]


def random_order(n: int, seed: int = 0):
    """Random ordering of n points: indices by ascending mix64(seed XOR i); returns the permutation."""
    perm = np.empty(max(int(n), 1), dtype=np.int64)
    rc = _load().oracle_random_order(int(n), ctypes.c_uint64(seed & (2 ** 64 - 1)), perm.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return perm[:n]


def mix64(z: int) -> int:
    """The splitmix64 finaliser of the ordering keys."""
    return int(_load().oracle_mix64(ctypes.c_uint64(z & (2 ** 64 - 1))))


def exact_loglik(locs, z, nu: float, theta) -> float:
    """Exact Gaussian log-likelihood of all points (dense Cholesky); z=None means y = 0."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(3)
    zz = None if z is None else np.ascontiguousarray(z, dtype=np.float64)
    out = np.zeros(1)
    rc = _load().oracle_exact_loglik(locs.ctypes.data, zz.ctypes.data if zz is not None else None, n, float(nu),
                                     th.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return float(out[0])


def kl_divergence(locs, nbr, m: int, nu: float, theta, threads: int = 0) -> float:
    """Eq. (9): exact minus Vecchia log-likelihood at y = 0."""
    n = np.asarray(locs).shape[0]
    return exact_loglik(locs, None, nu, theta) - loglik(locs, np.zeros(n), nbr, m, nu, theta, threads=threads)


def term_mp(locs, z, nbr, m: int, nu: float, theta, i: int, dps: int = 50) -> float:
    """l_i of Eq. (7) in arbitrary precision (mpmath, `dps` decimal digits), for adjudicating rounding
    differences between two FP64 evaluations of an ill-conditioned conditional.  The FP64 inputs are
    taken as exact; the covariance (Matern closed forms, nugget on equal indices), the Cholesky factor,
    the two forward solves and the univariate term follow the same steps as the C oracle."""
    import mpmath as mp

    locs = np.asarray(locs, dtype=np.float64)
    with mp.workdps(dps):
        s2, beta, tau2 = (mp.mpf(float(t)) for t in theta)
        k = int(min(i, m))
        J = [int(j) for j in np.asarray(nbr)[i, :k]]

        def cov(a, b):
            d = mp.sqrt((mp.mpf(locs[a, 0]) - mp.mpf(locs[b, 0])) ** 2 + (mp.mpf(locs[a, 1]) - mp.mpf(locs[b, 1])) ** 2)
            r = d / beta
            e = mp.exp(-r)
            if nu == 0.5:
                return s2 * e
            if nu == 1.5:
                return s2 * (1 + r) * e
            return s2 * (1 + r + r * r / 3) * e

        S = mp.matrix(k, k)
        for a in range(k):
            for b in range(a + 1):
                S[a, b] = S[b, a] = cov(J[a], J[b]) + (tau2 if a == b else 0)
        v = [cov(J[a], i) for a in range(k)]
        y = [mp.mpf(float(z[j])) for j in J]
        vp, yp = [], []
        if k:
            L = mp.cholesky(S)
            for r_ in range(k):
                av, ay = v[r_], y[r_]
                for q in range(r_):
                    av -= L[r_, q] * vp[q]
                    ay -= L[r_, q] * yp[q]
                vp.append(av / L[r_, r_])
                yp.append(ay / L[r_, r_])
        mu = mp.fsum(a * b for a, b in zip(vp, yp))
        c = s2 + tau2 - mp.fsum(a * a for a in vp)
        res = mp.mpf(float(z[i])) - mu
        return float(-(mp.log(2 * mp.pi) + mp.log(c) + res * res / c) / 2)
