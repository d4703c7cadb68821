"""Fixed nugget (Sigma + tau^2 I) against the oracle: covariance entries, l and
score, Fisher information, kriging; coincident locations become regular."""
import numpy as np
import pytest

import inputgen
from scorecheck import assert_score_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def exa():
    import paper_1908_06936_amd as exa

    return exa


def test_nugget_on_the_diagonal_only(orc, exa):
    x, y = inputgen.uniform(300, seed=41)
    x[7], y[7] = x[3], y[3]  # a coincident pair shares sigma^2 only
    th, t2 = [1.2, 0.1, 0.9], 0.35
    ctx = exa.Context(ts=256)
    ctx.set_nugget(t2)
    got = ctx.matern_cov(dev(x), dev(y), th).cpu().numpy()
    ref = orc.matern_cov_nugget(x, y, th, t2)
    np.testing.assert_allclose(got, ref, rtol=2e-13, atol=1e-300)
    assert got[3, 7] == th[0] and got[3, 3] == th[0] + t2


@pytest.mark.parametrize("n,ts,th,t2", [(700, 256, [1.0, 0.1, 0.8], 0.2), (1300, 512, [1.5, 0.05, 1.3], 0.01),
                                        (257, 128, [0.7, 0.2, 0.5], 1.5)])
def test_nugget_loglik_and_score_vs_oracle(orc, exa, n, ts, th, t2):
    x, y = inputgen.uniform(n, seed=300 + n)
    S = orc.matern_cov_nugget(x, y, th, t2)
    z = np.linalg.cholesky(S) @ inputgen.normals(n, seed=300 + n)
    ll_ref, g_ref = orc.loglik_grad_nugget(x, y, z, th, t2)
    ctx = exa.Context(ts=ts)
    ctx.set_nugget(t2)
    ll, g = ctx.loglik_grad(dev(x), dev(y), dev(z), th)
    assert ll == pytest.approx(ll_ref, rel=1e-10)
    assert_score_close(g, g_ref, n, th)
    assert ctx.loglik(dev(x), dev(y), dev(z), th) == pytest.approx(ll_ref, rel=1e-10)


def test_nugget_makes_coincident_locations_regular(orc, exa):
    x, y = inputgen.uniform(200, seed=5)
    x[10:20], y[10:20] = x[0:10], y[0:10]  # ten duplicated sites
    th, t2 = [1.0, 0.1, 1.0], 0.1
    z = inputgen.normals(200, seed=5)
    ctx = exa.Context(ts=128)
    ctx.set_nugget(t2)
    ll = ctx.loglik(dev(x), dev(y), dev(z), th)
    assert ll == pytest.approx(orc.loglik_grad_nugget(x, y, z, th, t2)[0], rel=1e-10)


def test_nugget_fisher_vs_oracle(orc, exa):
    n, th, t2 = 700, [1.0, 0.08, 0.9], 0.3
    x, y = inputgen.uniform(n, seed=77)
    ref = orc.fisher(x, y, th, nugget=t2)
    ctx = exa.Context(ts=256)
    ctx.set_nugget(t2)
    I = ctx.fisher(dev(x), dev(y), th)
    d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    print(f"max scaled error {np.max(np.abs(I - ref) / d):.2e}")
    assert np.max(np.abs(I - ref) / d) <= 1e-9
    ctx.set_nugget(0.0)
    assert np.max(np.abs(ctx.fisher(dev(x), dev(y), th) - orc.fisher(x, y, th)) / d) <= 1e-9


def test_nugget_predict_vs_oracle(orc, exa):
    n, m, th, t2 = 900, 200, [1.3, 0.1, 1.0], 0.25
    x, y = inputgen.uniform(n, seed=90)
    z = np.linalg.cholesky(orc.matern_cov_nugget(x, y, th, t2)) @ inputgen.normals(n, seed=90)
    xn, yn = inputgen.uniform(m, seed=91)
    xn[:5], yn[:5] = x[:5], y[:5]  # predictions at observed sites no longer interpolate
    ref_mean, ref_mse = orc.predict(x, y, z, th, xn, yn, nugget=t2)
    ctx = exa.Context(ts=256)
    ctx.set_nugget(t2)
    mean, mse = ctx.predict(dev(x), dev(y), dev(z), th, dev(xn), dev(yn))
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    assert np.abs(mean - ref_mean).max() <= 1e-9 * np.abs(z).max()
    assert np.abs(mse - ref_mse).max() <= 1e-9 * th[0]
    assert np.all(mse[:5] > 0.01 * t2)


def test_nugget_rejects_invalid(exa):
    ctx = exa.Context(ts=128)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(exa.ExaGeoError):
            ctx.set_nugget(bad)


def test_nugget_with_mixed_precision_and_great_circle(orc, exa):
    # the nugget sits on the FP64 diagonal tiles of the mixed factorisation,
    # and composes with the great-circle distance
    n, th, t2 = 700, [1.0, 0.05, 0.7], 0.2
    x, y = inputgen.uniform(n, seed=120)
    z = np.linalg.cholesky(orc.matern_cov_nugget(x, y, th, t2)) @ inputgen.normals(n, seed=120)
    ref = orc.loglik_grad_nugget(x, y, z, th, t2)[0]
    ctx = exa.Context(ts=128)
    ctx.set_nugget(t2)
    ctx.set_mixed_policy(0.0)
    got = ctx.loglik(dev(x), dev(y), dev(z), th, "mixed")
    assert got == pytest.approx(ref, rel=1e-6)
    u, v = inputgen.uniform(400, seed=121)
    lon, lat = 360.0 * u - 180.0, 150.0 * v - 75.0
    thg = [0.8, 900.0, 0.6]
    S = orc.matern_cov_gc(lon, lat, thg)
    S[np.diag_indices_from(S)] += t2
    L = np.linalg.cholesky(S)
    zg = L @ inputgen.normals(400, seed=121)
    ctx.set_distance("great_circle")
    assert ctx.loglik(dev(lon), dev(lat), dev(zg), thg) == pytest.approx(orc.loglik_from_factor(L, zg), rel=1e-10)
