"""Mixed-precision likelihood (FP64 diagonal tiles, FP32 / BF16 off-diagonal
tiles) against the FP64 oracle.

The mixed result is an approximation of eq. (2); its tests check
  * the plumbing exactly: when every off-diagonal tile is exactly zero (well
    separated clusters, one cluster per tile) the mixed and FP64 paths agree
    to FP64 rounding;
  * the error against the FP64 oracle stays within bounds set by the storage
    rounding of the off-diagonal covariances (unit roundoff 2^-24 for FP32 and
    2^-9 for BF16) amplified by the conditioning, measured on these inputs;
  * a wider BF16 band (fewer BF16 tiles) never does worse than a narrower
    one by more than rounding noise, and no BF16 tiles means FP32-only;
  * the mixed score (FP32 off-diagonal tiles of L^-1 and Sigma^-1, FP64
    diagonal tiles and sums) is exact when the off-diagonal tiles vanish and
    stays within measured bounds of the FP64 oracle otherwise.
"""
import math

import numpy as np
import pytest

import inputgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def exa():
    import paper_1908_06936_amd as exa

    return exa


def test_mixed_exact_when_off_diagonal_is_zero(orc, exa):
    # 4 clusters of exactly ts points at the corners of a square 2000 beta
    # wide: the location ordering keeps each cluster in one tile, so every
    # off-diagonal tile is exactly 0 in any precision
    ctx = exa.Context(ts=256, band_factor=3.0)
    x, y, lab = inputgen.corner_clusters(256, width=1.0, separation=200.0, seed=21)
    th = [1.0, 0.1, 1.0]
    z = np.zeros(x.size)
    ref = 0.0
    for c in range(4):
        m = lab == c
        z[m] = orc.simulate(x[m], y[m], th, inputgen.normals(256, seed=30 + c))
        ref += orc.loglik(x[m], y[m], z[m], th)
    X, Y, Z = dev(x), dev(y), dev(z)
    l64 = ctx.loglik(X, Y, Z, th, "fp64")
    lmx = ctx.loglik(X, Y, Z, th, "mixed")
    assert ctx.timings()["frac_bf16"] == 1.0  # all cross-cluster tiles far beyond the band
    assert l64 == pytest.approx(ref, rel=1e-12)
    assert lmx == pytest.approx(l64, rel=1e-12)


@pytest.mark.parametrize("beta,nu,tol", [(0.03, 0.5, 1e-7), (0.1, 0.5, 1e-6), (0.1, 1.0, 2e-5)])
def test_mixed_fp32_only_vs_oracle(orc, exa, beta, nu, tol):
    ctx = exa.Context(ts=256, band_factor=0.0)  # no BF16 tiles
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    ref = orc.loglik(x, y, z, th)
    got = ctx.loglik(dev(x), dev(y), dev(z), th, "mixed")
    tm = ctx.timings()
    assert tm["frac_bf16"] == 0.0 and tm["frac_fp32"] == 1.0
    rel = abs(got - ref) / abs(ref)
    print(f"FP32-only mixed: beta={beta} nu={nu} rel err {rel:.3e}")
    assert rel <= tol


@pytest.mark.parametrize("beta,nu,tol", [(0.03, 0.5, 1e-6), (0.1, 0.5, 1e-4), (0.1, 1.0, 2e-3)])
def test_mixed_bf16_band_vs_oracle(orc, exa, beta, nu, tol):
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    ref = orc.loglik(x, y, z, th)
    errs = {}
    for band in (3.0, 6.0, 1e9):
        ctx = exa.Context(ts=256, band_factor=band)
        st, got, _ = ctx.loglik_status(dev(x), dev(y), dev(z), th, "mixed")
        errs[band] = (abs(got - ref) / abs(ref) if st == exa.OK else math.inf, ctx.timings()["frac_bf16"], st)
    print(f"beta={beta} nu={nu}: " + ", ".join(f"band {b}: rel {e:.2e} bf16 {f:.2f} status {st}"
                                               for b, (e, f, st) in errs.items()))
    assert errs[1e9][1] == 0.0 and errs[1e9][2] == exa.OK
    # a wider band keeps more tiles in FP32
    assert errs[6.0][1] <= errs[3.0][1] and errs[3.0][1] > 0.0
    if nu == 0.5:
        assert errs[3.0][0] <= tol
    else:
        # nu = 1 on this grid: BF16 rounding of correlations near 0.1 can push
        # the smallest eigenvalue below zero; the library must then report a
        # failed pivot rather than a wrong number
        assert errs[3.0][2] == exa.ENOTPD or errs[3.0][0] <= tol


def test_mixed_gradient_deterministic(orc, exa):
    ctx = exa.Context(ts=256)
    x, y = inputgen.uniform(700, seed=3)
    th = [1.0, 0.1, 0.5]
    z = orc.simulate(x, y, th, inputgen.normals(700, seed=3))
    X, Y, Z = dev(x), dev(y), dev(z)
    a = ctx.loglik_grad(X, Y, Z, th, "mixed")
    b = ctx.loglik_grad(X, Y, Z, th, "mixed")
    assert a == b
    # the gradient call factors exactly as the l-only call does
    assert a[0] == ctx.loglik(X, Y, Z, th, "mixed")


def test_mixed_grad_exact_when_off_diagonal_is_zero(orc, exa):
    # every off-diagonal tile of L and of L^-1 is exactly zero: the FP32 parts
    # of the mixed gradient vanish and the FP64 diagonal parts remain
    ctx = exa.Context(ts=256, band_factor=3.0)
    x, y, lab = inputgen.corner_clusters(256, width=1.0, separation=200.0, seed=21)
    th = [1.0, 0.1, 1.0]
    z = np.zeros(x.size)
    gref = np.zeros(3)
    for c in range(4):
        m = lab == c
        z[m] = orc.simulate(x[m], y[m], th, inputgen.normals(256, seed=30 + c))
        gref += np.asarray(orc.loglik_grad(x[m], y[m], z[m], th)[1])
    X, Y, Z = dev(x), dev(y), dev(z)
    l64, g64 = ctx.loglik_grad(X, Y, Z, th, "fp64")
    lmx, gmx = ctx.loglik_grad(X, Y, Z, th, "mixed")
    assert lmx == pytest.approx(l64, rel=1e-12)
    np.testing.assert_allclose(g64, gref, rtol=1e-9, atol=1e-9 * np.abs(gref).max())
    np.testing.assert_allclose(gmx, g64, rtol=1e-11, atol=1e-11 * np.abs(g64).max())


# FP32 off-diagonal tiles of L, L^-1 and Sigma^-1: the score error against the
# FP64 oracle, relative to the largest score component (bounds measured on
# these inputs with a margin of about 10x: the error comes from the FP32
# factor, whose perturbation of Sigma the inverse amplifies)
@pytest.mark.parametrize("beta,nu,band,tol", [(0.03, 0.5, 0.0, 3e-6), (0.1, 0.5, 0.0, 1e-5), (0.03, 0.5, 3.0, 1e-5)])
def test_mixed_grad_vs_oracle(orc, exa, beta, nu, band, tol):
    ctx = exa.Context(ts=256, band_factor=band)
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    lref, gref = orc.loglik_grad(x, y, z, th)
    st, _, _ = ctx.loglik_status(dev(x), dev(y), dev(z), th, "mixed")
    assert st == exa.OK
    lmx, gmx = ctx.loglik_grad(dev(x), dev(y), dev(z), th, "mixed")
    gref = np.asarray(gref)
    err = np.abs(np.asarray(gmx) - gref) / np.abs(gref).max()
    print(f"mixed grad beta={beta} nu={nu} band={band}: l rel {abs(lmx - lref) / abs(lref):.2e}, "
          f"grad err / max|g| = {err}, g = {gmx}, ref = {list(gref)}")
    assert err.max() <= tol


def test_mixed_lbfgsb_mle_matches_fp64(orc, exa):
    ctx = exa.Context(ts=256, band_factor=0.0)
    x, y = inputgen.jittered_grid(30, seed=4)
    th = [1.0, 0.1, 0.5]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=4))
    X, Y, Z = dev(x), dev(y), dev(z)
    lb, ub, t0 = [0.01, 0.01, 0.1], [5.0, 2.0, 2.0], [0.5, 0.3, 0.5]
    th64, l64, s64 = ctx.mle(X, Y, Z, lb, ub, theta0=t0, tol=1e-7, method="lbfgsb", precision="fp64")
    thmx, lmx, smx = ctx.mle(X, Y, Z, lb, ub, theta0=t0, tol=1e-7, method="lbfgsb", precision="mixed")
    print("fp64", th64, l64, s64, "mixed", thmx, lmx, smx)
    assert smx["n_grad_evals"] > 0
    np.testing.assert_allclose(thmx, th64, rtol=2e-2)
    assert lmx == pytest.approx(l64, rel=1e-5)


def test_mixed_notpd_status(exa):
    ctx = exa.Context(ts=128)
    st, ll, info = ctx.loglik_status(dev([0.3, 0.3]), dev([0.2, 0.2]), dev([1.0, 0.5]), [4.0, 0.1, 0.5], "mixed")
    assert st == exa.ENOTPD and ll == -math.inf and info in (1, 2)


def test_mixed_all_fp64_band_reproduces_fp64_bitwise(orc, exa):
    # NT = 7: the band pool holds all 21 off-diagonal tiles, so every tile is
    # FP64 and the mixed path runs the FP64 arithmetic in the same order
    ctx = exa.Context(ts=256, band_factor=0.0, fp64_band=1e9)
    x, y = inputgen.jittered_grid(40, seed=5)
    th = [1.0, 0.1, 1.0]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=5))
    X, Y, Z = dev(x), dev(y), dev(z)
    l64 = ctx.loglik(X, Y, Z, th, "fp64")
    lmx = ctx.loglik(X, Y, Z, th, "mixed")
    tm = ctx.timings()
    assert tm["frac_fp64"] == 1.0 and tm["frac_bf16"] == 0.0
    assert lmx == l64
    assert l64 == pytest.approx(orc.loglik(x, y, z, th), rel=1e-10)


@pytest.mark.parametrize("beta,nu", [(0.1, 0.5), (0.1, 1.0)])
def test_mixed_fp64_band_reduces_error(orc, exa, beta, nu):
    # 60 x 60 grid, ts 128: NT = 29; the pool holds 4 NT = 116 of the 406
    # off-diagonal tiles, the closest ones
    x, y = inputgen.jittered_grid(60, seed=6)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=6))
    ref = orc.loglik(x, y, z, th)
    X, Y, Z = dev(x), dev(y), dev(z)
    errs = {}
    for fb in (0.0, 0.5):
        ctx = exa.Context(ts=128, band_factor=0.0, fp64_band=fb)
        st, got, _ = ctx.loglik_status(X, Y, Z, th, "mixed")
        errs[fb] = (abs(got - ref) / abs(ref) if st == exa.OK else math.inf, ctx.timings()["frac_fp64"])
    print(f"beta={beta} nu={nu}: " + ", ".join(f"fp64 band {b}: rel {e:.2e} (fp64 tiles {f:.2f})"
                                               for b, (e, f) in errs.items()))
    assert errs[0.0][1] == 0.0 and 0.0 < errs[0.5][1] <= 116 / 406 + 1e-12
    assert errs[0.5][0] < errs[0.0][0]


def test_mixed_grad_fp64_band_vs_oracle(orc, exa):
    # the FP64 band also sets the precision of the matching blocks of
    # Sigma^-1 (and of L): the score error drops against the FP32-only policy
    x, y = inputgen.jittered_grid(60, seed=6)
    th = [1.0, 0.1, 0.5]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=6))
    gref = np.asarray(orc.loglik_grad(x, y, z, th)[1])
    X, Y, Z = dev(x), dev(y), dev(z)
    errs = {}
    for fb in (0.0, 0.5):
        ctx = exa.Context(ts=128, band_factor=0.0, fp64_band=fb)
        g = np.asarray(ctx.loglik_grad(X, Y, Z, th, "mixed")[1])
        errs[fb] = (np.abs(g - gref) / np.abs(gref).max()).max()
    print(f"mixed score error / max|g|: FP32 only {errs[0.0]:.2e}, FP64 band 0.5 beta {errs[0.5]:.2e}")
    # measured 3.6e-6 and 2.8e-6: the band removes the largest terms of W's
    # error; the FP32 inverse factor outside it keeps the rest
    assert errs[0.5] < errs[0.0]
    assert errs[0.5] <= 1e-5


def test_mle_mixed_search_with_fp64_finish(exa):
    # 48 x 48 jittered grid, theta = (1, 0.1, 0.5): the mixed-precision search
    # followed by an FP64 finish reaches the FP64 L-BFGS-B optimum to 1e-6 of l
    import inputgen

    x, y = inputgen.jittered_grid(48, seed=4)
    n = x.size
    ctx = exa.Context(ts=256)
    th_true = [1.0, 0.1, 0.5]
    e = torch.as_tensor(inputgen.normals(n, seed=4), device="cuda")
    X, Y = dev(x), dev(y)
    Z = ctx.simulate(X, Y, th_true, e)
    lb, ub, th0 = [0.01, 0.01, 0.1], [5.0, 2.0, 3.0], [0.5, 0.3, 0.5]
    th64, ll64, st64 = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-7, method="lbfgsb", precision="fp64")
    ctx.set_mixed_policy(0.0)
    thm, llm, stm = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-7, method="lbfgsb_fp64_finish",
                            precision="mixed")
    print(f"fp64 {th64} {ll64} {st64}\nmixed+finish {thm} {llm} {stm}")
    assert st64["status"] == "OK" and stm["status"] == "OK"
    assert 0 < stm["n_fp64_finish_evals"] < stm["n_grad_evals"]
    # the reported value is an FP64 likelihood at the returned point
    assert ctx.loglik(X, Y, Z, thm) == llm
    assert abs(llm - ll64) <= 1e-6 * abs(ll64)
