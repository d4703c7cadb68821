"""CPU oracle for the exact Matern Gaussian log-likelihood (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it.

The numerics live in ``exageo_oracle.c`` (plain FP64 C, single-threaded per
dot product, optional OpenMP over independent rows with bitwise-identical
results).  This module is ctypes marshalling plus:

* ``mle``: maximises the oracle's l(theta) with SciPy's bounded optimisers (a
  library routine used as a step).  The paper's estimator is a bounded
  maximisation of eq. (2) over (sigma^2, beta, nu) started at the lower bound
  (Section 3, Example 2); the optimiser's internal steps are not part of the
  definition, so any correct bounded optimiser pins the maximiser.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exageo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOTPD = 0, -1, -2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP rows)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_besselk.restype = d
    lib.oracle_besselk.argtypes = [d, d]
    lib.oracle_besselk_scaled.restype = d
    lib.oracle_besselk_scaled.argtypes = [d, d]
    lib.oracle_besselk_dnu.restype = d
    lib.oracle_besselk_dnu.argtypes = [d, d]
    lib.oracle_besselk_dnu_scaled.restype = d
    lib.oracle_besselk_dnu_scaled.argtypes = [d, d]
    lib.oracle_digamma.restype = d
    lib.oracle_digamma.argtypes = [d]
    lib.oracle_matern.restype = d
    lib.oracle_matern.argtypes = [d, p]
    lib.oracle_matern_grad.restype = None
    lib.oracle_matern_grad.argtypes = [d, p, p]
    lib.oracle_matern_cov.restype = ctypes.c_int
    lib.oracle_matern_cov.argtypes = [i64, p, p, p, p]
    lib.oracle_matern_dcov.restype = ctypes.c_int
    lib.oracle_matern_dcov.argtypes = [i64, p, p, p, ctypes.c_int, p]
    lib.oracle_cholesky.restype = ctypes.c_int
    lib.oracle_cholesky.argtypes = [i64, p, p, p, p, p]
    lib.oracle_simulate.restype = ctypes.c_int
    lib.oracle_simulate.argtypes = [i64, p, p, p, p, p, p]
    lib.oracle_loglik.restype = ctypes.c_int
    lib.oracle_loglik.argtypes = [i64, p, p, p, p, p, p, p, p]
    lib.oracle_loglik_grad.restype = ctypes.c_int
    lib.oracle_loglik_grad.argtypes = [i64, p, p, p, p, p, p, p]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_num_threads.restype = None
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status: int, info: int = 0):
        super().__init__(f"oracle status {status} (info {info})")
        self.status = status
        self.info = info


def set_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def besselk(nu: float, x: float) -> float:
    return float(_load().oracle_besselk(float(nu), float(x)))


def besselk_scaled(nu: float, x: float) -> float:
    """e^x K_nu(x)."""
    return float(_load().oracle_besselk_scaled(float(nu), float(x)))


def besselk_dnu(nu: float, x: float) -> float:
    return float(_load().oracle_besselk_dnu(float(nu), float(x)))


def besselk_dnu_scaled(nu: float, x: float) -> float:
    return float(_load().oracle_besselk_dnu_scaled(float(nu), float(x)))


def digamma(z: float) -> float:
    return float(_load().oracle_digamma(float(z)))


def matern(r: float, theta) -> float:
    th = _f64(theta)
    return float(_load().oracle_matern(float(r), _ptr(th)))


def matern_grad(r: float, theta) -> np.ndarray:
    th = _f64(theta)
    out = np.zeros(3)
    _load().oracle_matern_grad(float(r), _ptr(th), _ptr(out))
    return out


def matern_cov(x, y, theta) -> np.ndarray:
    x, y, th = _f64(x), _f64(y), _f64(theta)
    n = x.size
    cov = np.empty((n, n))
    st = _load().oracle_matern_cov(n, _ptr(x), _ptr(y), _ptr(th), _ptr(cov))
    if st:
        raise OracleError(st)
    return cov


def matern_dcov(x, y, theta, comp: int) -> np.ndarray:
    """Dense matrix of dSigma/dtheta_comp (comp 0: sigma^2, 1: beta, 2: nu)."""
    x, y, th = _f64(x), _f64(y), _f64(theta)
    n = x.size
    out = np.empty((n, n))
    st = _load().oracle_matern_dcov(n, _ptr(x), _ptr(y), _ptr(th), int(comp), _ptr(out))
    if st:
        raise OracleError(st)
    return out


def fisher(x, y, theta, nugget: float = 0.0) -> np.ndarray:
    """Fisher information of theta = (sigma^2, beta, nu) for the zero-mean
    Gaussian field observed at (x, y) (the exact_fisher function of the
    package's API table, Section 3): the expected negative Hessian of eq. (2),
        I_jk = tr(Sigma^-1 dSigma_j Sigma^-1 dSigma_k) / 2.
    With A_j = Sigma^-1 dSigma_j (a library solve used as a step) the trace is
    the sum of the elementwise product of A_j and A_k^T.  A fixed nugget tau^2
    adds tau^2 I to Sigma and nothing to its theta-derivatives."""
    x, y, th = _f64(x), _f64(y), _f64(theta)
    S = matern_cov_nugget(x, y, th, nugget)
    A = [np.linalg.solve(S, matern_dcov(x, y, th, k)) for k in range(3)]
    I = np.empty((3, 3))
    for j in range(3):
        for k in range(3):
            I[j, k] = 0.5 * np.sum(A[j] * A[k].T)
    return I


def matern_cov_nugget(x, y, theta, nugget: float) -> np.ndarray:
    """Sigma(theta) + tau^2 I: the Matern covariance (eq. 3) of a field observed
    with independent noise of variance tau^2 (the nugget effect the package's
    kernels can include, Section 6); coincident distinct locations share sigma^2,
    only each observation's own variance gains tau^2."""
    S = matern_cov(x, y, theta)
    if nugget:
        S[np.diag_indices_from(S)] += nugget
    return S


def loglik_grad_nugget(x, y, z, theta, nugget: float):
    """(l, grad l) of eq. (2) for Sigma(theta) + tau^2 I with tau^2 fixed:
    dense library factorisation and inverse as steps,
        g_k = a^T dSigma_k a / 2 - tr(Sigma^-1 dSigma_k) / 2,  a = Sigma^-1 z
    (the nugget is constant in theta, so the derivative matrices are those of
    the Matern part)."""
    x, y, z, th = _f64(x), _f64(y), _f64(z), _f64(theta)
    S = matern_cov_nugget(x, y, th, nugget)
    ll = loglik_from_factor(np.linalg.cholesky(S), z)
    Si = np.linalg.inv(S)
    a = Si @ z
    grad = np.empty(3)
    for k in range(3):
        dS = matern_dcov(x, y, th, k)
        grad[k] = 0.5 * a @ dS @ a - 0.5 * np.sum(Si * dS)
    return ll, grad


def cholesky_packed(x, y, theta) -> np.ndarray:
    """Packed lower (row-major) Cholesky factor of Sigma(theta)."""
    x, y, th = _f64(x), _f64(y), _f64(theta)
    n = x.size
    L = np.empty(n * (n + 1) // 2)
    info = ctypes.c_int64(0)
    st = _load().oracle_cholesky(n, _ptr(x), _ptr(y), _ptr(th), _ptr(L), ctypes.byref(info))
    if st:
        raise OracleError(st, info.value)
    return L


def simulate(x, y, theta, e) -> np.ndarray:
    """z = L e, L = chol(Sigma(theta)): one draw of the zero-mean field."""
    x, y, th, e = _f64(x), _f64(y), _f64(theta), _f64(e)
    n = x.size
    z = np.empty(n)
    info = ctypes.c_int64(0)
    st = _load().oracle_simulate(n, _ptr(x), _ptr(y), _ptr(th), _ptr(e), _ptr(z), ctypes.byref(info))
    if st:
        raise OracleError(st, info.value)
    return z


def unpack_lower(Lp: np.ndarray, n: int) -> np.ndarray:
    """Dense lower-triangular matrix from the packed row-major factor."""
    L = np.zeros((n, n))
    L[np.tril_indices(n)] = Lp
    return L


def predict(x, y, z, theta, xn, yn, nugget: float = 0.0):
    """Kriging at new locations (the conditional distribution of the Gaussian
    field given the data, paper Section 4 and Section 5): with c_i the vector
    of covariances between new point i and the observed points,
        mean_i = c_i^T Sigma^-1 z,   mse_i = sigma^2 - c_i^T Sigma^-1 c_i,
    evaluated through the oracle's own Cholesky factor L (Sigma = L L^T) as
    (L^-1 c_i)^T (L^-1 z) and sigma^2 - |L^-1 c_i|^2; the triangular solves are
    a library routine used as a step.  With a nugget tau^2 the observations
    carry independent noise: Sigma gains tau^2 I (factored by LAPACK), c_i does
    not (the prediction is of the noise-free field).  Returns (mean, mse)."""
    import scipy.linalg

    x, y, z, th, xn, yn = _f64(x), _f64(y), _f64(z), _f64(theta), _f64(xn), _f64(yn)
    n, m = x.size, xn.size
    if nugget:
        L = np.linalg.cholesky(matern_cov_nugget(x, y, th, nugget))
    else:
        L = unpack_lower(cholesky_packed(x, y, th), n)
    S = matern_cov(np.concatenate([x, xn]), np.concatenate([y, yn]), th)
    C = S[:n, n:]
    v = scipy.linalg.solve_triangular(L, z, lower=True)
    V = scipy.linalg.solve_triangular(L, C, lower=True)
    return V.T @ v, th[0] - np.sum(V * V, axis=0)


def morton_order(x, y) -> np.ndarray:
    """Z-order of the locations: coordinates scaled to [0, 65536) over their
    bounding box, truncated to 16 bits, bits interleaved (x in the even bits),
    ties by index.  This is the ordering whose consecutive runs of ts points
    form the tiles of the diagonal-super-tile (DST) variant."""
    x, y = _f64(x), _f64(y)
    wx, wy = x.max() - x.min(), y.max() - y.min()
    sx = 65535.999 / wx if wx > 0 else 0.0
    sy = 65535.999 / wy if wy > 0 else 0.0
    qx = ((x - x.min()) * sx).astype(np.uint64)
    qy = ((y - y.min()) * sy).astype(np.uint64)
    code = np.zeros(x.size, dtype=np.uint64)
    for b in range(16):
        code |= ((qx >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        code |= ((qy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return np.lexsort((np.arange(x.size), code))


def dst_covariance(x, y, theta, ts: int, band: int):
    """The DST approximation (paper Section 2.1, Fig. 1(b)): Sigma(theta) of
    the locations in Z-order, cut into tiles of ts points, with every tile
    (I, J), |I - J| >= band, set to zero.  Returns (Sigma_DST, order)."""
    order = morton_order(x, y)
    xs, ys = _f64(x)[order], _f64(y)[order]
    S = matern_cov(xs, ys, theta)
    t = np.arange(xs.size) // ts
    S[np.abs(t[:, None] - t[None, :]) >= band] = 0.0
    return S, order


def loglik_dst(x, y, z, theta, ts: int, band: int) -> float:
    """eq. (2) with Sigma replaced by its DST approximation; the factorisation
    is a library routine used as a step."""
    S, order = dst_covariance(x, y, theta, ts, band)
    return loglik_from_factor(np.linalg.cholesky(S), _f64(z)[order])


def loglik_grad_dst(x, y, z, theta, ts: int, band: int):
    """(l, grad l) of the DST likelihood: g_k = a^T dS_k a / 2 - tr(S^-1 dS_k) / 2
    with S the DST covariance, dS_k its derivative (the derivative of eq. (3)
    on the kept tiles, zero elsewhere) and a = S^-1 z."""
    S, order = dst_covariance(x, y, theta, ts, band)
    xs, ys, zs = _f64(x)[order], _f64(y)[order], _f64(z)[order]
    n = xs.size
    L = np.linalg.cholesky(S)
    ll = loglik_from_factor(L, zs)
    Si = np.linalg.inv(S)
    a = Si @ zs
    t = np.arange(n) // ts
    dS = np.zeros((3, n, n))
    for i in range(n):
        for j in range(i + 1):
            if abs(t[i] - t[j]) >= band:
                continue
            r = float(np.hypot(xs[i] - xs[j], ys[i] - ys[j]))
            g = matern_grad(r, theta)
            dS[:, i, j] = g
            dS[:, j, i] = g
    grad = np.array([0.5 * a @ dS[k] @ a - 0.5 * np.sum(Si * dS[k]) for k in range(3)])
    return ll, grad


EARTH_RADIUS_KM = 6371.0


def great_circle(lon1, lat1, lon2, lat2):
    """Great-circle distance in km on a sphere of radius 6371 between
    (longitude, latitude) points in degrees (haversine, central angle by
    atan2 as in Veness 2010)."""
    p1, p2 = np.radians(lat1), np.radians(lat2)
    dp, dl = p2 - p1, np.radians(np.asarray(lon2) - np.asarray(lon1))
    a = np.sin(dp / 2) ** 2 + np.cos(p1) * np.cos(p2) * np.sin(dl / 2) ** 2
    a = np.clip(a, 0.0, 1.0)
    return EARTH_RADIUS_KM * 2.0 * np.arctan2(np.sqrt(a), np.sqrt(1.0 - a))


def matern_cov_gc(lon, lat, theta) -> np.ndarray:
    """eq. (3) with great-circle distances (the dmetric option, Section 3)."""
    lon, lat = _f64(lon), _f64(lat)
    n = lon.size
    D = great_circle(lon[:, None], lat[:, None], lon[None, :], lat[None, :])
    S = np.empty((n, n))
    for i in range(n):
        for j in range(i + 1):
            S[i, j] = S[j, i] = matern(D[i, j], theta)
    return S


def _dcov_gc(lon, lat, theta) -> np.ndarray:
    """The three theta-derivative matrices of eq. (3) with great-circle distances."""
    lon, lat = _f64(lon), _f64(lat)
    n = lon.size
    D = great_circle(lon[:, None], lat[:, None], lon[None, :], lat[None, :])
    dS = np.zeros((3, n, n))
    for i in range(n):
        for j in range(i + 1):
            g = matern_grad(D[i, j], theta)
            dS[:, i, j] = g
            dS[:, j, i] = g
    return dS


def fisher_gc(lon, lat, theta) -> np.ndarray:
    """Fisher information (as `fisher`) with great-circle distances."""
    S = matern_cov_gc(lon, lat, theta)
    dS = _dcov_gc(lon, lat, theta)
    A = [np.linalg.solve(S, dS[k]) for k in range(3)]
    return np.array([[0.5 * np.sum(A[j] * A[k].T) for k in range(3)] for j in range(3)])


def predict_gc(lon, lat, z, theta, lon_new, lat_new):
    """Kriging (as `predict`) with great-circle distances; library Cholesky and
    triangular solves as steps."""
    import scipy.linalg

    lon, lat, z = _f64(lon), _f64(lat), _f64(z)
    n = lon.size
    S = matern_cov_gc(np.concatenate([lon, _f64(lon_new)]), np.concatenate([lat, _f64(lat_new)]), theta)
    L = np.linalg.cholesky(S[:n, :n])
    v = scipy.linalg.solve_triangular(L, z, lower=True)
    V = scipy.linalg.solve_triangular(L, S[:n, n:], lower=True)
    return V.T @ v, _f64(theta)[0] - np.sum(V * V, axis=0)


def loglik_grad_gc(lon, lat, z, theta):
    """(l, grad l) with great-circle distances; dense factorisation and inverse
    by library routines."""
    lon, lat, z = _f64(lon), _f64(lat), _f64(z)
    n = lon.size
    S = matern_cov_gc(lon, lat, theta)
    ll = loglik_from_factor(np.linalg.cholesky(S), z)
    Si = np.linalg.inv(S)
    a = Si @ z
    D = great_circle(lon[:, None], lat[:, None], lon[None, :], lat[None, :])
    dS = np.zeros((3, n, n))
    for i in range(n):
        for j in range(i + 1):
            g = matern_grad(D[i, j], theta)
            dS[:, i, j] = g
            dS[:, j, i] = g
    grad = np.array([0.5 * a @ dS[k] @ a - 0.5 * np.sum(Si * dS[k]) for k in range(3)])
    return ll, grad


def dense_factor_lapack(x, y, theta) -> np.ndarray:
    """Lower Cholesky factor of the oracle's own dense Sigma(theta) (eq. 3) by
    LAPACK (numpy): the plain definition with a library factorisation as a
    step, for the full-size checks where the unblocked O(n^3) loop is slow."""
    return np.linalg.cholesky(matern_cov(x, y, theta))


def loglik_from_factor(L: np.ndarray, z) -> float:
    """eq. (2) from a lower Cholesky factor: -(n ln 2 pi + 2 sum ln L_ii + |L^-1 z|^2) / 2."""
    import scipy.linalg

    z = _f64(z)
    v = scipy.linalg.solve_triangular(L, z, lower=True)
    return -0.5 * (z.size * np.log(2.0 * np.pi) + 2.0 * np.log(np.diag(L)).sum() + v @ v)


def loglik(x, y, z, theta, *, details: bool = False):
    """l(theta) of eq. (2); raises OracleError on invalid input / non-PD."""
    x, y, z, th = _f64(x), _f64(y), _f64(z), _f64(theta)
    n = x.size
    ll, ld, q = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    info = ctypes.c_int64(0)
    st = _load().oracle_loglik(n, _ptr(x), _ptr(y), _ptr(z), _ptr(th), ctypes.byref(ll),
                               ctypes.byref(ld), ctypes.byref(q), ctypes.byref(info))
    if st:
        raise OracleError(st, info.value)
    if details:
        return ll.value, ld.value, q.value
    return ll.value


def loglik_status(x, y, z, theta):
    """(status, loglik, info) without raising."""
    x, y, z, th = _f64(x), _f64(y), _f64(z), _f64(theta)
    n = x.size
    ll = ctypes.c_double(0)
    info = ctypes.c_int64(0)
    st = _load().oracle_loglik(n, _ptr(x), _ptr(y), _ptr(z), _ptr(th), ctypes.byref(ll),
                               None, None, ctypes.byref(info))
    return st, ll.value, info.value


def loglik_grad(x, y, z, theta):
    """(l, grad) with grad = dl/d(sigma^2, beta, nu)."""
    x, y, z, th = _f64(x), _f64(y), _f64(z), _f64(theta)
    n = x.size
    ll = ctypes.c_double(0)
    g = np.zeros(3)
    info = ctypes.c_int64(0)
    st = _load().oracle_loglik_grad(n, _ptr(x), _ptr(y), _ptr(z), _ptr(th), ctypes.byref(ll),
                                    _ptr(g), ctypes.byref(info))
    if st:
        raise OracleError(st, info.value)
    return ll.value, g


def mle(x, y, z, lb, ub, theta0=None, *, use_grad: bool = True, tol: float = 1e-9,
        max_evals: int = 2000):
    """Bounded maximiser of the oracle's l(theta) (SciPy L-BFGS-B or Powell).

    Non-PD points are infeasible: the objective returns +inf there (the
    optimiser then backs off), matching the reading that a singular Sigma has
    l = -inf.
    """
    from scipy.optimize import minimize

    lb, ub = _f64(lb), _f64(ub)
    th0 = _f64(lb if theta0 is None else theta0)

    def f(t):
        st, ll, _ = loglik_status(x, y, z, t)
        return -ll if st == OK else np.inf

    def fg(t):
        try:
            ll, g = loglik_grad(x, y, z, t)
        except OracleError:
            return 1e300, np.zeros(3)
        return -ll, -g

    bounds = list(zip(lb, ub))
    if use_grad:
        res = minimize(fg, th0, jac=True, method="L-BFGS-B", bounds=bounds,
                       options={"ftol": tol, "gtol": 1e-10, "maxfun": max_evals})
    else:
        res = minimize(f, th0, method="Powell", bounds=bounds,
                       options={"ftol": tol, "xtol": 1e-10, "maxfev": max_evals})
    return np.asarray(res.x), -float(res.fun), int(res.nfev)
