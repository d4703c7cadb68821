"""Fisher information (exageo_fisher) against the oracle, the Markov closed
form at full size, and properties that hold at any size."""
import numpy as np
import pytest

import inputgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# entry (j, k) is compared relative to sqrt(I_jj I_kk), the natural scale of
# the matrix; B_j = L^-1 dSigma_j L^-T goes through the explicit inverse, so
# its rounding grows with the condition of L (about 1e4 here)
TOL = 1e-9


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def exa():
    import paper_1908_06936_amd as exa

    return exa


def _err(I, ref):
    d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    return np.max(np.abs(I - ref) / d)


@pytest.mark.parametrize("n,ts,th", [(700, 256, [1.0, 0.1, 0.8]), (1000, 384, [1.5, 0.05, 1.3]),
                                     (300, 128, [0.8, 0.2, 0.5]), (100, 128, [1.2, 0.07, 2.1]),
                                     (1300, 512, [0.6, 0.03, 0.9]), (256, 128, [1.0, 0.1, 1.0])])
def test_fisher_vs_oracle(orc, exa, n, ts, th):
    # several tiles with a ragged last one, a single padded tile (n = 100)
    x, y = inputgen.uniform(n, seed=200 + n)
    ref = orc.fisher(x, y, th)
    ctx = exa.Context(ts=ts)
    I = ctx.fisher(dev(x), dev(y), th)
    print(f"n={n} ts={ts}: max scaled error {_err(I, ref):.2e}")
    assert _err(I, ref) <= TOL
    np.testing.assert_array_equal(I, I.T)


def test_fisher_single_point(exa):
    # n = 1: only sigma^2 is identifiable, I = diag(1 / (2 sigma^4), 0, 0)
    ctx = exa.Context(ts=128)
    I = ctx.fisher(dev([0.3]), dev([0.4]), [1.5, 0.1, 0.8])
    ref = np.zeros((3, 3))
    ref[0, 0] = 1.0 / (2 * 1.5 ** 2)
    np.testing.assert_allclose(I, ref, rtol=1e-15, atol=0)


def test_fisher_ignores_precision_policy_and_rejects_dst(orc, exa):
    n, th = 600, [1.1, 0.06, 1.0]
    x, y = inputgen.uniform(n, seed=7)
    ctx = exa.Context(ts=128)
    I0 = ctx.fisher(dev(x), dev(y), th)
    ctx.set_mixed_policy(3.0, fp64_band=1.0)
    assert np.array_equal(ctx.fisher(dev(x), dev(y), th), I0)
    ctx.set_dst_band(2)
    with pytest.raises(exa.ExaGeoError):
        ctx.fisher(dev(x), dev(y), th)
    ctx.set_dst_band(0)
    assert np.array_equal(ctx.fisher(dev(x), dev(y), th), I0)


def test_fisher_not_positive_definite(exa):
    # two coincident locations make Sigma singular
    x = np.array([0.1, 0.1, 0.5, 0.9])
    y = np.array([0.2, 0.2, 0.4, 0.7])
    ctx = exa.Context(ts=128)
    with pytest.raises(exa.NotPositiveDefinite):
        ctx.fisher(dev(x), dev(y), [1.0, 0.1, 0.5])


def test_fisher_markov_full_size(exa):
    # nu = 1/2 on a line at n = 40,000 with tile 768: the (sigma^2, beta) block
    # has the closed form of the Markov chain's factorised density,
    #   I = e e^T / (2 s2^2) + sum_i [s2 grad(rho_i) grad(rho_i)^T / v_i + grad(ln v_i) grad(ln v_i)^T / 2]
    n, s2, beta = 40000, 1.2, 0.1
    t, y0 = inputgen.collinear(n, mean_gap=0.004, seed=77)
    d = np.diff(np.sort(t))
    rho = np.exp(-d / beta)
    drho = np.stack([np.zeros_like(rho), rho * d / beta ** 2])
    dlnv = np.stack([np.full_like(rho, 1.0 / s2), -2.0 * rho * drho[1] / (1.0 - rho ** 2)])
    v = s2 * (1.0 - rho ** 2)
    ref = np.zeros((2, 2))
    ref[0, 0] = 0.5 / s2 ** 2
    ref += s2 * (drho / v) @ drho.T + 0.5 * dlnv @ dlnv.T
    ctx = exa.Context(ts=768)
    I = ctx.fisher(dev(t), dev(y0), [s2, beta, 0.5])
    print(f"I[:2,:2] {I[:2, :2].tolist()} ref {ref.tolist()}")
    assert _err(I[:2, :2], ref) <= 1e-8
    assert np.all(np.linalg.eigvalsh(I) > 0)


def test_fisher_config4_size(exa):
    # n = 90,000 (300 x 300 jittered grid), tile 768: the derivative matrices
    # live in the workspace as lower tiles (n^2 / 2 doubles each); checks that
    # hold at any size: I_ss = n / (2 sigma^4), I_sk = -g_k / sigma^2 against
    # the score at z = 0, symmetry and positive definiteness
    x, y = inputgen.jittered_grid(300, seed=0)
    n, th = x.size, [1.0, 0.1, 0.5]
    ctx = exa.Context(ts=768)
    ctx.set_profiling(True)
    I = ctx.fisher(dev(x), dev(y), th)
    tm = ctx.timings()
    print(f"n={n}: I = {I.tolist()}, {tm['total_ms']:.0f} ms, products {tm['fisher_flops'] / (tm['grad_ms'] * 1e-3) / 1e12:.1f} TFLOP/s")
    _, g = ctx.loglik_grad(dev(x), dev(y), dev(np.zeros(n)), th)
    assert I[0, 0] == n / (2 * th[0] ** 2)
    np.testing.assert_allclose(I[0, 1:], -np.asarray(g[1:]) / th[0], rtol=1e-9)
    np.testing.assert_array_equal(I, I.T)
    assert np.all(np.linalg.eigvalsh(I) > 0)


def test_fisher_variance_row_is_the_score_trace_at_full_size(exa):
    # at any size: I_ss = n / (2 sigma^4), and with z = 0 the score is
    # g_k = -tr(Sigma^-1 dSigma_k) / 2, so I_sk = -g_k / sigma^2 (the score runs
    # through the fused LAUUM contraction, a different path from the products here)
    n, th = 40000, [1.0, 0.1, 1.0]
    x, y = inputgen.jittered_grid(200, seed=3)
    ctx = exa.Context(ts=768)
    I = ctx.fisher(dev(x), dev(y), th)
    _, g = ctx.loglik_grad(dev(x), dev(y), dev(np.zeros(n)), th)
    assert I[0, 0] == n / (2 * th[0] ** 2)
    np.testing.assert_allclose(I[0, 1:], -np.asarray(g[1:]) / th[0], rtol=1e-9)
    assert np.all(np.linalg.eigvalsh(I) > 0)
