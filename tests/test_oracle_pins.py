"""Pins of the CPU oracle against closed forms, library routines and invariants.

Every pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them:

* special functions: DLMF closed forms, asymptotes and recurrences, and
  mpmath/scipy evaluated independently;
* Matern covariance (paper eq. 3): the exponential (nu = 1/2) and the
  nu = 3/2, 5/2 closed forms, the r = 0 limit;
* log-likelihood (paper eq. 2, mu = 0): hand-derived n = 1, 2, 3 values, an
  independent numpy/scipy dense evaluation, the exact O(n) likelihood of the
  one-dimensional exponential (Markov) model, block additivity and
  permutation / scaling / variance-profile invariances;
* gradient: the variance closed form (q - n) / (2 sigma^2), an independent
  numpy evaluation at nu = 1/2 through the exponential-integral form of
  dK/dnu, and central differences.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import inputgen

LN2PI = math.log(2.0 * math.pi)


# --------------------------------------------------------------- Bessel K_nu
@pytest.mark.parametrize("x", [1e-6, 0.01, 0.3, 1.0, 1.2, 1.25, 1.3, 2.0, 7.5, 40.0, 300.0, 700.0])
def test_besselk_half_integer_closed_forms(orc, x):
    # DLMF 10.39.2 and the order recurrence DLMF 10.29.1
    k12 = math.sqrt(math.pi / (2 * x))  # scaled by e^x
    assert orc.besselk_scaled(0.5, x) == pytest.approx(k12, rel=4e-15)
    assert orc.besselk_scaled(1.5, x) == pytest.approx(k12 * (1 + 1 / x), rel=4e-15)
    assert orc.besselk_scaled(2.5, x) == pytest.approx(k12 * (1 + 3 / x + 3 / x ** 2), rel=4e-15)
    assert orc.besselk_scaled(-1.5, x) == orc.besselk_scaled(1.5, x)  # DLMF 10.27.3


def test_besselk_against_mpmath(orc):
    import mpmath as mp

    mp.mp.dps = 30
    worst = 0.0
    for nu in [0.001, 0.05, 0.3, 0.49, 0.77, 1.0, 1.2, 2.0, 2.3, 3.7, 5.0]:
        for x in [1e-8, 1e-3, 0.05, 0.5, 1.0, 1.249, 1.25, 1.6, 3.0, 12.0, 90.0, 650.0]:
            ref = float(mp.besselk(nu, x) * mp.e ** x)
            worst = max(worst, abs(orc.besselk_scaled(nu, x) / ref - 1))
    assert worst < 1e-14


def test_besselk_known_value_and_scipy(orc):
    # K_1(1) (Abramowitz & Stegun Table 9.8) and scipy's kv as a library routine
    assert orc.besselk(1.0, 1.0) == pytest.approx(0.6019072301972346, rel=1e-15)
    for nu in [0.25, 0.8, 1.7]:
        for x in [0.1, 1.0, 4.0, 25.0]:
            assert orc.besselk(nu, x) == pytest.approx(sp.kv(nu, x), rel=1e-13)


def test_besselk_small_x_asymptote(orc):
    # K_nu(x) ~ Gamma(nu)/2 (x/2)^-nu as x -> 0 (DLMF 10.30.2), relative
    # correction O(x^(2 min(nu, 1 - nu))) for 0 < nu < 1, O(x^2 log x) above
    x = 1e-12
    for nu in [0.6, 1.7, 3.2]:
        asym = 0.5 * math.gamma(nu) * (x / 2) ** (-nu)
        assert orc.besselk(nu, x) == pytest.approx(asym, rel=1e-8)


def test_besselk_recurrence_across_methods(orc):
    # K_{nu+1} - K_{nu-1} = (2 nu / x) K_nu (DLMF 10.29.1), evaluated by
    # independent calls on both sides of the series / recurrence split
    for nu in [0.3, 1.1, 2.7]:
        for x in [0.7, 1.24, 1.26, 3.0, 40.0]:
            lhs = orc.besselk_scaled(nu + 1, x) - orc.besselk_scaled(nu - 1, x)
            rhs = 2 * nu / x * orc.besselk_scaled(nu, x)
            assert lhs == pytest.approx(rhs, rel=2e-14)


def test_besselk_large_x_asymptote(orc):
    # DLMF 10.40.2 with a_k(nu) of DLMF 10.17.1:
    # e^x K_nu(x) sqrt(2x/pi) ~ sum_k a_k(nu) / x^k,
    # a_k = (4nu^2 - 1^2)(4nu^2 - 3^2)...(4nu^2 - (2k-1)^2) / (k! 8^k)
    x = 600.0
    for nu in [0.2, 1.0, 2.2]:
        m = 4 * nu * nu
        series, a = 1.0, 1.0
        for k in range(1, 10):
            a *= (m - (2 * k - 1) ** 2) / (k * 8.0)
            series += a / x ** k
        assert orc.besselk_scaled(nu, x) * math.sqrt(2 * x / math.pi) == pytest.approx(series, rel=2e-15)


# ---------------------------------------------------------------- dK/dnu
@pytest.mark.parametrize("x,ref", [(1.0, 0.16659724500287904), (0.01, 42.467586459386496),
                                   (5.0, 3.4579931158389626e-4)])
def test_dnu_half_closed_form_values(orc, x, ref):
    # dK_nu/dnu at nu = 1/2 equals sqrt(pi/(2x)) E1(2x) e^x (DLMF 10.38.7)
    closed = math.sqrt(math.pi / (2 * x)) * sp.exp1(2 * x) * math.exp(x)
    assert closed == pytest.approx(ref, rel=1e-14)
    assert orc.besselk_dnu(0.5, x) == pytest.approx(closed, rel=5e-15)


def test_dnu_against_mpmath_and_parity(orc):
    import mpmath as mp

    mp.mp.dps = 30
    for nu in [0.05, 0.7, 1.0, 2.3, 4.0]:
        for x in [1e-5, 0.2, 1.3, 6.0, 80.0]:
            ref = float(mp.diff(lambda v: mp.besselk(v, x), nu) * mp.e ** x)
            assert orc.besselk_dnu_scaled(nu, x) == pytest.approx(ref, rel=1e-14)
    # K is even in nu, so dK/dnu is odd and vanishes at nu = 0
    assert orc.besselk_dnu_scaled(0.0, 0.7) == 0.0
    assert orc.besselk_dnu_scaled(-0.8, 0.7) == -orc.besselk_dnu_scaled(0.8, 0.7)


# ---------------------------------------------------------------- digamma
def test_digamma(orc):
    g = 0.5772156649015329
    assert orc.digamma(1.0) == pytest.approx(-g, rel=1e-15)                      # DLMF 5.4.12
    assert orc.digamma(0.5) == pytest.approx(-g - 2 * math.log(2), rel=1e-15)   # DLMF 5.4.13
    for z in [0.003, 0.4, 1.7, 9.99, 10.0, 55.0]:
        assert orc.digamma(z) == pytest.approx(sp.digamma(z), rel=1e-14, abs=1e-15)
        assert orc.digamma(z + 1) - orc.digamma(z) == pytest.approx(1 / z, rel=1e-13)


# ---------------------------------------------------------------- Matern (eq. 3)
@pytest.mark.parametrize("r", [1e-7, 0.003, 0.05, 0.2, 0.9, 5.0, 60.0])
def test_matern_closed_forms(orc, r):
    s2, beta = 1.7, 0.13
    x = r / beta
    assert orc.matern(r, [s2, beta, 0.5]) == pytest.approx(s2 * math.exp(-x), rel=3e-15, abs=1e-300)
    assert orc.matern(r, [s2, beta, 1.5]) == pytest.approx(s2 * (1 + x) * math.exp(-x), rel=3e-15, abs=1e-300)
    assert orc.matern(r, [s2, beta, 2.5]) == pytest.approx(s2 * (1 + x + x * x / 3) * math.exp(-x),
                                                          rel=3e-15, abs=1e-300)


def test_matern_limits_and_scipy(orc):
    th = [2.0, 0.1, 1.3]
    assert orc.matern(0.0, th) == 2.0
    assert orc.matern(1e-12, th) == pytest.approx(2.0, rel=1e-9)
    assert orc.matern(200.0, th) == 0.0  # x = 2000: underflows to exactly 0
    rs = np.linspace(1e-4, 3, 200)
    vals = np.array([orc.matern(r, th) for r in rs])
    assert np.all(np.diff(vals) < 0)  # strictly decreasing in r
    for r in [0.01, 0.1, 0.4]:
        x = r / th[1]
        ref = th[0] * 2 ** (1 - th[2]) / math.gamma(th[2]) * x ** th[2] * sp.kv(th[2], x)
        assert orc.matern(r, th) == pytest.approx(ref, rel=1e-13)


def test_matern_grad_closed_forms_and_fd(orc):
    s2, beta = 1.4, 0.2
    for r in [0.01, 0.15, 0.6]:
        x = r / beta
        d = orc.matern_grad(r, [s2, beta, 0.5])
        assert d[0] == pytest.approx(math.exp(-x), rel=1e-14)
        assert d[1] == pytest.approx(s2 * x * math.exp(-x) / beta, rel=1e-14)
        # nu-derivative at 1/2 from DLMF 10.38.7 and psi(1/2) = -g - 2 ln 2
        c = math.sqrt(2.0 / math.pi)
        dk = math.sqrt(math.pi / (2 * x)) * sp.exp1(2 * x) * math.exp(x)
        dnu = s2 * math.exp(-x) * (-math.log(2) - sp.digamma(0.5) + math.log(x)) \
            + s2 * c * math.sqrt(x) * dk
        assert d[2] == pytest.approx(dnu, rel=1e-12)
    th = np.array([1.1, 0.07, 1.3])
    for r in [0.02, 0.1, 0.3]:
        d = orc.matern_grad(r, th)
        for k in range(3):
            h = 1e-6 * th[k]
            tp, tm = th.copy(), th.copy()
            tp[k] += h
            tm[k] -= h
            fd = (orc.matern(r, tp) - orc.matern(r, tm)) / (2 * h)
            assert d[k] == pytest.approx(fd, rel=1e-7)
    assert list(orc.matern_grad(0.0, th)) == [1.0, 0.0, 0.0]


# ---------------------------------------------------------------- l(theta) (eq. 2)
def test_loglik_n1(orc):
    s2, z = 2.0, 0.7
    ref = -0.5 * (LN2PI + math.log(s2) + z * z / s2)
    assert ref == pytest.approx(-1.3880121234846454, rel=1e-15)
    assert orc.loglik([0.0], [0.0], [z], [s2, 0.1, 0.5]) == pytest.approx(ref, rel=1e-15)


def test_loglik_n2_exponential(orc):
    # rho = exp(-r/beta); det = s2^2 (1 - rho^2); quadratic form by the 2x2 inverse
    s2, beta, r = 1.0, 0.1, 0.1
    rho = math.exp(-r / beta)
    z1, z2 = 1.0, 0.5
    ref = -0.5 * (2 * LN2PI + math.log(s2 ** 2 * (1 - rho ** 2))
                  + (z1 ** 2 - 2 * rho * z1 * z2 + z2 ** 2) / (s2 * (1 - rho ** 2)))
    assert ref == pytest.approx(-2.2752643321336263, rel=1e-15)
    got = orc.loglik([0, 0.1], [0, 0], [z1, z2], [s2, beta, 0.5])
    assert got == pytest.approx(ref, rel=1e-14)


def test_loglik_n3_cofactors(orc):
    # nu = 3/2 closed-form covariance; determinant and inverse by cofactors
    xs, ys = [0.0, 0.1, 0.0], [0.0, 0.0, 0.2]
    s2, beta = 1.5, 0.1
    z = np.array([1.0, -0.5, 0.25])

    def c(r):
        x = r / beta
        return s2 * (1 + x) * math.exp(-x)

    r01, r02, r12 = 0.1, 0.2, math.hypot(0.1, 0.2)
    a, b, cc = c(r01), c(r02), c(r12)
    assert (a, b, cc) == pytest.approx((1.103638323514327, 0.6090087745647572, 0.518796349096766), rel=1e-14)
    d = s2
    det = d * (d * d - cc * cc) - a * (a * d - cc * b) + b * (a * cc - d * b)
    cof = np.array([[d * d - cc * cc, -(a * d - b * cc), a * cc - b * d],
                    [-(a * d - cc * b), d * d - b * b, -(d * cc - a * b)],
                    [a * cc - d * b, -(d * cc - b * a), d * d - a * a]])
    q = z @ (cof / det) @ z
    ref = -0.5 * (3 * LN2PI + math.log(det) + q)
    assert ref == pytest.approx(-4.325813976873814, rel=1e-14)
    assert orc.loglik(xs, ys, z, [s2, beta, 1.5]) == pytest.approx(ref, rel=1e-14)


def _dense_loglik_scipy(x, y, z, th):
    """Independent dense evaluation: scipy.special.kv covariance + numpy LAPACK."""
    s2, beta, nu = th
    r = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    xx = r / beta
    with np.errstate(invalid="ignore", divide="ignore"):
        C = s2 * 2 ** (1 - nu) / sp.gamma(nu) * xx ** nu * sp.kv(nu, xx)
    C[r == 0] = s2
    sign, logdet = np.linalg.slogdet(C)
    assert sign > 0
    q = z @ np.linalg.solve(C, z)
    return -0.5 * (x.size * LN2PI + logdet + q), C


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.7])
def test_loglik_vs_independent_dense(orc, nu):
    x, y = inputgen.jittered_grid(20, seed=3)
    th = [1.0, 0.1, nu]
    e = inputgen.normals(x.size, seed=3)
    z = orc.simulate(x, y, th, e)
    ref, _ = _dense_loglik_scipy(x, y, z, th)
    assert orc.loglik(x, y, z, th) == pytest.approx(ref, rel=1e-11)


def test_loglik_markov_exact_1d(orc):
    # nu = 1/2 on a line is a Markov (Ornstein-Uhlenbeck) process: the joint
    # density factorises into N(z1; 0, s2) prod N(z_i; rho_i z_{i-1}, s2 (1 - rho_i^2)).
    n, s2, beta = 1500, 1.3, 0.1
    t, y0 = inputgen.collinear(n, mean_gap=0.005, seed=11)
    rho = np.exp(-np.diff(t) / beta)
    e = inputgen.normals(n, seed=11)
    z = np.empty(n)
    z[0] = math.sqrt(s2) * e[0]
    for i in range(1, n):  # exact sequential sampling of the same process
        z[i] = rho[i - 1] * z[i - 1] + math.sqrt(s2 * (1 - rho[i - 1] ** 2)) * e[i]
    v = s2 * (1 - rho ** 2)
    ref = -0.5 * (LN2PI + math.log(s2) + z[0] ** 2 / s2)
    ref += np.sum(-0.5 * (LN2PI + np.log(v) + (z[1:] - rho * z[:-1]) ** 2 / v))
    perm = inputgen.shuffled(n, seed=1)  # the oracle must not depend on the order
    assert orc.loglik(t[perm], y0[perm], z[perm], [s2, beta, 0.5]) == pytest.approx(ref, rel=1e-12)


def test_loglik_block_additivity(orc):
    x, y, lab = inputgen.clusters(60, 3, width=0.3, separation=1000.0, seed=5)
    th = [1.0, 0.1, 0.9]
    z = inputgen.normals(x.size, seed=5)
    total = orc.loglik(x, y, z, th)
    parts = sum(orc.loglik(x[lab == c], y[lab == c], z[lab == c], th) for c in range(3))
    assert total == pytest.approx(parts, rel=1e-13)


def test_loglik_invariances(orc):
    x, y = inputgen.uniform(150, seed=2)
    z = inputgen.normals(150, seed=2)
    th = np.array([1.2, 0.15, 0.8])
    ll, logdet, q = orc.loglik(x, y, z, th, details=True)
    perm = inputgen.shuffled(150, seed=2)
    assert orc.loglik(x[perm], y[perm], z[perm], th) == pytest.approx(ll, rel=1e-12)
    c = 3.7  # scaling locations and range together leaves Sigma unchanged
    assert orc.loglik(c * x, c * y, z, [th[0], c * th[1], th[2]]) == pytest.approx(ll, rel=1e-12)
    # variance profile: Sigma = s2 R  ->  l(s2) = -1/2 (n ln 2pi + n ln s2 + logdet R + q_R / s2)
    _, logdet_r, q_r = orc.loglik(x, y, z, [1.0, th[1], th[2]], details=True)
    n = x.size
    for s2 in [0.3, 4.0]:
        ref = -0.5 * (n * LN2PI + n * math.log(s2) + logdet_r + q_r / s2)
        assert orc.loglik(x, y, z, [s2, th[1], th[2]]) == pytest.approx(ref, rel=1e-13)


# ---------------------------------------------------------------- gradient
def test_grad_variance_closed_form(orc):
    x, y = inputgen.jittered_grid(12, seed=4)
    th = [1.6, 0.12, 1.2]
    z = inputgen.normals(x.size, seed=4)
    ll, _, q = orc.loglik(x, y, z, th, details=True)
    ll2, g = orc.loglik_grad(x, y, z, th)
    assert ll2 == ll
    assert g[0] == pytest.approx((q - x.size) / (2 * th[0]), rel=1e-11)


def test_grad_independent_dense_at_half(orc):
    # g_k = 1/2 a^T D_k a - 1/2 tr(Sigma^-1 D_k) with numpy inverse and the
    # nu = 1/2 derivative through E1 (DLMF 10.38.7): independent of the oracle
    x, y = inputgen.jittered_grid(14, seed=6)
    s2, beta, nu = 1.3, 0.09, 0.5
    z = inputgen.normals(x.size, seed=6)
    ll_ref, C = _dense_loglik_scipy(x, y, z, [s2, beta, nu])
    r = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    xx = r / beta
    off = r > 0
    D0 = C / s2
    D1 = np.zeros_like(C)
    D1[off] = s2 * xx[off] * np.exp(-xx[off]) / beta
    D2 = np.zeros_like(C)
    dk = np.sqrt(np.pi / (2 * xx[off])) * sp.exp1(2 * xx[off]) * np.exp(xx[off])
    D2[off] = C[off] * (-math.log(2) - sp.digamma(0.5) + np.log(xx[off])) \
        + s2 * math.sqrt(2 / math.pi) * np.sqrt(xx[off]) * dk
    W = np.linalg.inv(C)
    a = W @ z
    gref = [0.5 * a @ D @ a - 0.5 * np.sum(W * D) for D in (D0, D1, D2)]
    ll, g = orc.loglik_grad(x, y, z, [s2, beta, nu])
    assert ll == pytest.approx(ll_ref, rel=1e-11)
    for k in range(3):
        assert g[k] == pytest.approx(gref[k], rel=1e-9, abs=1e-9 * abs(gref[1]))


def test_grad_central_differences(orc):
    x, y = inputgen.jittered_grid(10, seed=8)
    th = np.array([0.9, 0.11, 1.4])
    e = inputgen.normals(x.size, seed=8)
    z = orc.simulate(x, y, th, e)
    _, g = orc.loglik_grad(x, y, z, th)
    for k in range(3):
        h = 1e-5 * th[k]
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (orc.loglik(x, y, z, tp) - orc.loglik(x, y, z, tm)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6)


# ---------------------------------------------------------------- error statuses
def test_statuses(orc):
    x, y = inputgen.uniform(30, seed=1)
    z = inputgen.normals(30, seed=1)
    th = [1.0, 0.1, 0.5]
    # two coincident locations first, sigma^2 = 4: the second pivot is
    # 4 - (4/2)^2 = 0 exactly, so the factorisation stops at column 2
    x2, y2 = x.copy(), y.copy()
    x2[1], y2[1] = x2[0], y2[0]
    st, ll, info = orc.loglik_status(x2, y2, z, [4.0, 0.1, 0.5])
    assert st == orc.ENOTPD and ll == -math.inf and info == 2
    # the paper's upper bounds nu = beta = 5 on a unit-square grid give a
    # covariance that is singular to working precision
    xg, yg = inputgen.jittered_grid(20, seed=0)
    st, ll, info = orc.loglik_status(xg, yg, inputgen.normals(400), [1.0, 5.0, 5.0])
    assert st == orc.ENOTPD and info > 1
    for bad in ([0.0, 0.1, 0.5], [1.0, -0.1, 0.5], [1.0, 0.1, 0.0], [math.nan, 0.1, 0.5]):
        st, _, _ = orc.loglik_status(x, y, z, bad)
        assert st == orc.EINVAL
    z2 = z.copy()
    z2[3] = math.nan
    assert orc.loglik_status(x, y, z2, th)[0] == orc.EINVAL


# ---------------------------------------------------------------- MLE (bounded)
def test_mle_interior_stationary(orc):
    x, y = inputgen.jittered_grid(20, seed=0)
    th_true = [1.0, 0.1, 0.5]
    z = orc.simulate(x, y, th_true, inputgen.normals(x.size, seed=0))
    lb, ub = [0.01, 0.01, 0.01], [5.0, 5.0, 5.0]
    th, ll, nev = orc.mle(x, y, z, lb, ub, theta0=[0.5, 0.3, 0.7])
    assert ll >= orc.loglik(x, y, z, th_true)
    _, g = orc.loglik_grad(x, y, z, th)
    interior = [(lb[k] * 1.01 < th[k] < ub[k] * 0.99) for k in range(3)]
    for k in range(3):
        if interior[k]:
            assert abs(g[k]) * th[k] < 1e-3 * abs(ll)
    # sigma^2 at the maximiser is the profile value q_R(beta, nu) / n
    _, _, q_r = orc.loglik(x, y, z, [1.0, th[1], th[2]], details=True)
    assert th[0] == pytest.approx(q_r / x.size, rel=1e-3)


def test_lapack_factor_path_matches_unblocked_oracle(orc):
    # the full-size helper (oracle covariance + library Cholesky) agrees with
    # the oracle's own unblocked factorisation on a case both can do
    import inputgen

    x, y = inputgen.jittered_grid(15, seed=3)
    th = [1.3, 0.08, 0.9]
    z = inputgen.normals(x.size, seed=3)
    L = orc.dense_factor_lapack(x, y, th)
    assert orc.loglik_from_factor(L, z) == pytest.approx(orc.loglik(x, y, z, th), rel=1e-12)


# ------------------------------------------------------------- kriging pins
def test_predict_interpolates_the_data(orc):
    # the conditional expectation at an observed location is the observation,
    # with zero variance
    import inputgen

    x, y = inputgen.uniform(120, seed=40)
    th = [1.7, 0.2, 1.3]
    z = orc.simulate(x, y, th, inputgen.normals(120, seed=40))
    idx = np.array([0, 7, 55, 119])
    mean, mse = orc.predict(x, y, z, th, x[idx], y[idx])
    np.testing.assert_allclose(mean, z[idx], rtol=1e-9, atol=1e-9)
    assert np.all(np.abs(mse) <= 1e-8 * th[0])


def test_predict_far_away_reverts_to_the_prior(orc):
    import inputgen

    x, y = inputgen.uniform(80, seed=41)
    th = [2.5, 0.05, 0.8]
    z = orc.simulate(x, y, th, inputgen.normals(80, seed=41))
    mean, mse = orc.predict(x, y, z, th, np.array([60.0]), np.array([-40.0]))
    assert abs(mean[0]) < 1e-300 and mse[0] == pytest.approx(th[0], rel=1e-15)


def test_predict_markov_closed_form(orc):
    # nu = 1/2 on a line: the exponential covariance is Markov, so kriging
    # uses only the two neighbours of the new point (one beyond the ends):
    #   w_a = r_a (1 - r_b^2) / (1 - r_a^2 r_b^2),  w_b = r_b (1 - r_a^2) / (1 - r_a^2 r_b^2),
    #   mse = s2 (1 - w_a r_a - w_b r_b),  r = exp(-distance / beta)
    rng = np.random.default_rng(42)
    s = np.sort(rng.uniform(0.0, 3.0, 60))
    x, y = s, np.zeros_like(s)
    th = [1.4, 0.35, 0.5]
    z = orc.simulate(x, y, th, rng.standard_normal(60))
    q = np.array([-0.4, 0.71, 1.505, 2.2, 3.3])
    mean, mse = orc.predict(x, y, z, th, q, np.zeros_like(q))
    for k, p in enumerate(q):
        if p < s[0] or p > s[-1]:
            j = 0 if p < s[0] else len(s) - 1
            r = np.exp(-abs(p - s[j]) / th[1])
            em, ev = r * z[j], th[0] * (1.0 - r * r)
        else:
            b = np.searchsorted(s, p)
            a = b - 1
            ra, rb = np.exp(-(p - s[a]) / th[1]), np.exp(-(s[b] - p) / th[1])
            d = 1.0 - ra * ra * rb * rb
            wa, wb = ra * (1.0 - rb * rb) / d, rb * (1.0 - ra * ra) / d
            em, ev = wa * z[a] + wb * z[b], th[0] * (1.0 - wa * ra - wb * rb)
        assert mean[k] == pytest.approx(em, rel=1e-10, abs=1e-12)
        assert mse[k] == pytest.approx(ev, rel=1e-9, abs=1e-12)


# --------------------------------------------------------------- DST pins
def test_dst_band_covering_all_tiles_is_exact(orc):
    import inputgen

    x, y = inputgen.uniform(300, seed=70)
    th = [1.1, 0.15, 0.9]
    z = orc.simulate(x, y, th, inputgen.normals(300, seed=70))
    assert orc.loglik_dst(x, y, z, th, 64, 5) == pytest.approx(orc.loglik(x, y, z, th), rel=1e-12)


def test_dst_single_band_is_block_diagonal(orc):
    # band 1 keeps only the diagonal tiles: l is the sum of the exact
    # likelihoods of the tiles' point sets
    import inputgen

    x, y = inputgen.uniform(300, seed=71)
    th = [0.9, 0.2, 1.4]
    z = orc.simulate(x, y, th, inputgen.normals(300, seed=71))
    order = orc.morton_order(x, y)
    ref = sum(orc.loglik(x[order[s:s + 64]], y[order[s:s + 64]], z[order[s:s + 64]], th) for s in range(0, 300, 64))
    assert orc.loglik_dst(x, y, z, th, 64, 1) == pytest.approx(ref, rel=1e-12)


def test_morton_order_is_a_z_curve(orc):
    # the four quadrants of the unit square come in Z order (lower-left,
    # lower-right, upper-left, upper-right), recursively
    x = np.array([0.1, 0.9, 0.1, 0.9, 0.2, 0.3])
    y = np.array([0.1, 0.1, 0.9, 0.9, 0.05, 0.2])
    order = orc.morton_order(x, y)
    assert list(order[-3:]) == [1, 2, 3]
    assert set(order[:3]) == {0, 4, 5}


def test_dst_gradient_matches_differences(orc):
    import inputgen

    x, y = inputgen.uniform(90, seed=72)
    th = np.array([1.2, 0.04, 0.8])
    z = orc.simulate(x, y, th, inputgen.normals(90, seed=72))
    _, g = orc.loglik_grad_dst(x, y, z, th, 32, 2)
    for k in range(3):
        h = 1e-6 * th[k]
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (orc.loglik_dst(x, y, z, tp, 32, 2) - orc.loglik_dst(x, y, z, tm, 32, 2)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6)


# -------------------------------------------------- great-circle distance pins
def test_great_circle_closed_forms(orc):
    R = orc.EARTH_RADIUS_KM
    assert orc.great_circle(0.0, 0.0, 90.0, 0.0) == pytest.approx(R * np.pi / 2, rel=1e-14)
    assert orc.great_circle(10.0, 90.0, -70.0, -90.0) == pytest.approx(R * np.pi, rel=1e-14)
    assert orc.great_circle(30.0, 0.0, 30.0, 45.0) == pytest.approx(R * np.pi / 4, rel=1e-14)
    assert orc.great_circle(179.5, 0.0, -179.5, 0.0) == pytest.approx(R * np.radians(1.0), rel=1e-12)
    assert orc.great_circle(12.0, -33.0, 12.0, -33.0) == 0.0


def test_great_circle_small_patch_matches_planar(orc):
    # on a patch of 1e-3 degrees at the equator the sphere is flat to ~1e-13:
    # the likelihood equals the Euclidean one in km
    import inputgen

    u, v = inputgen.uniform(120, seed=80)
    lon, lat = 1e-3 * u, 1e-3 * v
    km = orc.EARTH_RADIUS_KM * np.radians(1.0)
    th = [1.3, 0.02, 0.9]
    z = orc.simulate(lon * km, lat * km, th, inputgen.normals(120, seed=80))
    l_gc, _ = orc.loglik_grad_gc(lon, lat, z, th)
    assert l_gc == pytest.approx(orc.loglik(lon * km, lat * km, z, th), rel=1e-9)


def test_great_circle_likelihood_is_rotation_invariant(orc):
    import inputgen

    u, v = inputgen.uniform(60, seed=81)
    lon, lat = 360.0 * u - 180.0, 160.0 * v - 80.0
    th = [1.0, 3000.0, 0.7]
    S = orc.matern_cov_gc(lon, lat, th)
    z = np.linalg.cholesky(S) @ inputgen.normals(60, seed=81)
    l0, g0 = orc.loglik_grad_gc(lon, lat, z, th)
    l1, g1 = orc.loglik_grad_gc(lon + 77.0, lat, z, th)
    assert l1 == pytest.approx(l0, rel=1e-12)
    np.testing.assert_allclose(g1, g0, rtol=1e-9)


# ------------------------------------------------------- Fisher information
def test_fisher_variance_entry_and_symmetry(orc):
    # dSigma/dsigma^2 = Sigma / sigma^2, so I_ss = n / (2 sigma^4) exactly and
    # I_sk = tr(Sigma^-1 dSigma_k) / (2 sigma^2); the matrix is symmetric PD.
    x, y = inputgen.uniform(150, seed=91)
    th = np.array([1.7, 0.08, 1.3])
    I = orc.fisher(x, y, th)
    assert I[0, 0] == pytest.approx(150 / (2 * th[0] ** 2), rel=1e-10)
    S = orc.matern_cov(x, y, th)
    for k in (1, 2):
        tr = np.trace(np.linalg.solve(S, orc.matern_dcov(x, y, th, k)))
        assert I[0, k] == pytest.approx(tr / (2 * th[0]), rel=1e-9)
    np.testing.assert_allclose(I, I.T, rtol=1e-9)
    assert np.all(np.linalg.eigvalsh(I) > 0)


def test_fisher_markov_closed_form(orc):
    # nu = 1/2 on a line: z_1 ~ N(0, s2), z_i | z_{i-1} ~ N(rho_i z_{i-1}, v_i),
    # rho_i = exp(-d_i / beta), v_i = s2 (1 - rho_i^2).  The information adds
    # over the factors; a Gaussian factor N(m z', v) with E z'^2 = s2 carries
    # s2 grad(m) grad(m)^T / v + grad(ln v) grad(ln v)^T / 2.
    n, s2, beta = 300, 0.9, 0.07
    t, y0 = inputgen.collinear(n, mean_gap=0.01, seed=5)
    d = np.diff(np.sort(t))
    rho = np.exp(-d / beta)
    drho = np.stack([np.zeros_like(rho), rho * d / beta ** 2])
    dlnv = np.stack([np.full_like(rho, 1.0 / s2), -2.0 * rho * drho[1] / (1.0 - rho ** 2)])
    v = s2 * (1.0 - rho ** 2)
    ref = np.zeros((2, 2))
    ref[0, 0] = 0.5 / s2 ** 2
    ref += s2 * (drho / v) @ drho.T + 0.5 * dlnv @ dlnv.T
    I = orc.fisher(t, y0, [s2, beta, 0.5])
    np.testing.assert_allclose(I[:2, :2], ref, rtol=1e-9)


def test_fisher_is_the_hessian_of_the_expected_loglik(orc):
    # I(theta0) = -Hessian of f(theta) = E_theta0[l(theta)]
    #           = -(ln det Sigma(theta) + tr(Sigma(theta)^-1 Sigma(theta0))) / 2 + const,
    # which needs only covariance values: central second differences pin every
    # entry, the nu row included, independently of the derivative matrices.
    x, y = inputgen.uniform(120, seed=17)
    th0 = np.array([1.2, 0.09, 0.9])
    S0 = orc.matern_cov(x, y, th0)

    def f(th):
        S = orc.matern_cov(x, y, th)
        return -0.5 * (np.linalg.slogdet(S)[1] + np.trace(np.linalg.solve(S, S0)))

    def hess(rel):
        h = rel * th0
        H = np.empty((3, 3))
        for j in range(3):
            for k in range(3):
                ej, ek = np.eye(3)[j] * h[j], np.eye(3)[k] * h[k]
                H[j, k] = (f(th0 + ej + ek) - f(th0 + ej - ek) - f(th0 - ej + ek)
                           + f(th0 - ej - ek)) / (4 * h[j] * h[k])
        return H

    H = (4 * hess(1e-3) - hess(2e-3)) / 3  # Richardson: O(h^4)
    I = orc.fisher(x, y, th0)
    scale = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    assert np.max(np.abs(-H - I) / scale) < 1e-7


# ------------------------------------------------------------------- nugget
def test_nugget_zero_is_the_unblocked_oracle(orc):
    x, y = inputgen.uniform(180, seed=33)
    th = [1.1, 0.09, 1.3]
    z = orc.simulate(x, y, th, inputgen.normals(180, seed=33))
    l0, g0 = orc.loglik_grad(x, y, z, th)
    l1, g1 = orc.loglik_grad_nugget(x, y, z, th, 0.0)
    assert l1 == pytest.approx(l0, rel=1e-12)
    np.testing.assert_allclose(g1, g0, rtol=1e-9)


def test_nugget_white_noise_limit(orc):
    # beta so small that every off-diagonal covariance underflows: Sigma = (s2 + t2) I
    s2, t2 = 1.3, 0.4
    x, y = inputgen.jittered_grid(10, seed=2)
    z = inputgen.normals(x.size, seed=2)
    th = [s2, 1e-5, 0.5]
    v = s2 + t2
    ll, g = orc.loglik_grad_nugget(x, y, z, th, t2)
    assert ll == pytest.approx(-0.5 * (x.size * (LN2PI + math.log(v)) + z @ z / v), rel=1e-13)
    # d/dsigma^2 = (|z|^2 / v - n) / (2 v); the range and smoothness have no effect
    assert g[0] == pytest.approx((z @ z / v - x.size) / (2 * v), rel=1e-12)
    assert g[1] == 0.0 and g[2] == 0.0
    I = orc.fisher(x, y, th, nugget=t2)
    assert I[0, 0] == pytest.approx(x.size / (2 * v * v), rel=1e-12)


def test_nugget_gradient_central_differences(orc):
    x, y = inputgen.uniform(120, seed=8)
    th, t2 = np.array([0.9, 0.12, 0.7]), 0.25
    z = orc.simulate(x, y, th, inputgen.normals(120, seed=8))
    _, g = orc.loglik_grad_nugget(x, y, z, th, t2)
    for k in range(3):
        h = 1e-6 * th[k]
        e = np.eye(3)[k] * h
        fd = (orc.loglik_grad_nugget(x, y, z, th + e, t2)[0] - orc.loglik_grad_nugget(x, y, z, th - e, t2)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_nugget_fisher_is_the_hessian_of_the_expected_loglik(orc):
    x, y = inputgen.uniform(100, seed=19)
    th0, t2 = np.array([1.0, 0.1, 1.1]), 0.3
    S0 = orc.matern_cov_nugget(x, y, th0, t2)

    def f(th):
        S = orc.matern_cov_nugget(x, y, th, t2)
        return -0.5 * (np.linalg.slogdet(S)[1] + np.trace(np.linalg.solve(S, S0)))

    def hess(rel):
        h = rel * th0
        H = np.empty((3, 3))
        for j in range(3):
            for k in range(3):
                ej, ek = np.eye(3)[j] * h[j], np.eye(3)[k] * h[k]
                H[j, k] = (f(th0 + ej + ek) - f(th0 + ej - ek) - f(th0 - ej + ek)
                           + f(th0 - ej - ek)) / (4 * h[j] * h[k])
        return H

    H = (4 * hess(1e-3) - hess(2e-3)) / 3
    I = orc.fisher(x, y, th0, nugget=t2)
    scale = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    assert np.max(np.abs(-H - I) / scale) < 1e-7
    # the variance entry no longer has the nugget-free closed form
    assert abs(I[0, 0] - x.size / (2 * th0[0] ** 2)) > 1e-3 * I[0, 0]


def test_nugget_predict_single_observation(orc):
    # one observation z at s: mean at s = s2 z / (s2 + t2), mse = s2 t2 / (s2 + t2)
    s2, t2, z = 1.4, 0.6, 0.9
    mean, mse = orc.predict([0.3], [0.4], [z], [s2, 0.1, 0.8], [0.3], [0.4], nugget=t2)
    assert mean[0] == pytest.approx(s2 * z / (s2 + t2), rel=1e-14)
    assert mse[0] == pytest.approx(s2 * t2 / (s2 + t2), rel=1e-14)


def test_great_circle_fisher_and_kriging(orc):
    # Fisher: the variance entry n / (2 sigma^4) and invariance under a rotation
    # in longitude; kriging: interpolation of the data and the prior at the
    # antipode of a small cluster
    u, v = inputgen.uniform(50, seed=61)
    lon, lat = 40.0 * u - 20.0, 30.0 * v + 10.0
    th = [1.3, 800.0, 0.8]
    I = orc.fisher_gc(lon, lat, th)
    assert I[0, 0] == pytest.approx(50 / (2 * th[0] ** 2), rel=1e-10)
    np.testing.assert_allclose(orc.fisher_gc(lon + 123.0, lat, th), I, rtol=1e-9)
    z = np.linalg.cholesky(orc.matern_cov_gc(lon, lat, th)) @ inputgen.normals(50, seed=61)
    mean, mse = orc.predict_gc(lon, lat, z, th, lon[:5], lat[:5])
    np.testing.assert_allclose(mean, z[:5], rtol=1e-9, atol=1e-9)
    assert np.abs(mse).max() <= 1e-9
    mean, mse = orc.predict_gc(lon, lat, z, th, [180.0], [-25.0])
    assert abs(mean[0]) < 1e-8 and mse[0] == pytest.approx(th[0], rel=1e-12)  # correlations there ~ e^-22


@pytest.mark.slow
def test_theta_recovery_with_fisher_standard_errors(orc):
    # 16 simulated fields on a 15 x 15 jittered grid, theta = (1, 0.1, 0.5):
    # the oracle's maximisers, standardised by the Fisher-information standard
    # errors at the truth, have medians near 0 and spreads near 1 (a wrong
    # score sign or a Fisher information off by a factor of 3 fails this)
    x, y = inputgen.jittered_grid(15, seed=0)
    th = np.array([1.0, 0.1, 0.5])
    se = np.sqrt(np.diag(np.linalg.inv(orc.fisher(x, y, th))))
    zs = []
    for r in range(1, 17):
        z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=r))
        thh, _, _ = orc.mle(x, y, z, [0.01, 0.01, 0.05], [5.0, 2.0, 3.0], theta0=[0.8, 0.15, 0.6])
        zs.append((thh - th) / se)
    zs = np.array(zs)
    assert np.all(np.abs(np.median(zs, axis=0)) < 1.5)
    assert np.all((zs.std(axis=0) > 0.6) & (zs.std(axis=0) < 1.8))
