"""Mixed precision (FP64 diagonal tiles; each off-diagonal tile FP64, FP32 or
BF16 by the precision map) against the FP64 oracle, the FP64 path and exact
closed forms.

Claimed, and asserted at the stated tolerance |dl| / |l| <= 1e-6:
  * the library's default map (by correlation: FP64 tiles whose correlation
    bound is >= 0.3, BF16 below 1e-4 together with their updates, FP32
    otherwise; one FP64 refinement step of Sigma^-1 z), within the range of
    the benchmark fields (nu <= 1, beta <= 0.1 on the unit square), on 40 x 40 jittered
    grids and uniform points against the oracle, on the 1-D Markov line at
    n = 40,000 with tile 768 against its O(n) closed form (all three tile
    precisions present), and on the 200 x 200 jittered grid at n = 40,000
    against the FP64 path (itself pinned to the oracle at 1e-10);
  * the plumbing exactly: with every off-diagonal tile zero, mixed and FP64
    agree to rounding; with every tile FP64 and no refinement the mixed path
    is the FP64 path bitwise.
Not claimed (the distance bands of BF16 beyond 3 beta, FP32 only, the map
without refinement, and the default map on smoother, longer-range fields such
as nu = 1.5, beta = 0.2, where it measured 1.3e-6): their errors are printed
for the record, and only
structural facts (tile fractions, statuses) are asserted.  A mixed
factorisation that fails is reported as ENOTPD with l = -inf (status tests).
"""
import math

import numpy as np
import pytest

import inputgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LN2PI = math.log(2 * math.pi)
CLAIM = 1e-6


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def exa():
    import paper_1908_06936_amd as exa

    return exa


def rel(a, b):
    return abs(a - b) / abs(b)


# ------------------------------------------------------------ plumbing
@pytest.mark.parametrize("dist_policy", [False, True])
def test_mixed_exact_when_off_diagonal_is_zero(orc, exa, dist_policy):
    # 4 clusters of exactly ts points at the corners of a square 2000 beta
    # wide: the location ordering keeps each cluster in one tile, so every
    # off-diagonal tile is exactly 0 in any precision
    ctx = exa.Context(ts=256, band_factor=3.0) if dist_policy else exa.Context(ts=256)
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
    assert ctx.timings()["frac_bf16"] == 1.0  # all cross-cluster tiles far beyond either rule
    assert l64 == pytest.approx(ref, rel=1e-12)
    assert lmx == pytest.approx(l64, rel=1e-12)


def test_mixed_all_fp64_reproduces_fp64_bitwise(orc, exa):
    # NT = 7: the pool holds all 21 off-diagonal tiles; with every tile FP64
    # and no refinement the mixed path runs the FP64 arithmetic in FP64 order
    ctx = exa.Context(ts=256)
    ctx.set_mixed_correlation(0.0, 0.0)
    ctx.set_mixed_refinement(0)
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
    # the gradient: with every tile on the FP64 band the mixed inverse factor
    # and its LAUUM are FP64 throughout (band kernels for every off-diagonal
    # tile, other blocking and order than the FP64 path: equal to rounding)
    l64g, g64 = ctx.loglik_grad(X, Y, Z, th, "fp64")
    lmxg, gmx = ctx.loglik_grad(X, Y, Z, th, "mixed")
    assert lmxg == lmx and l64g == l64
    g64, gmx = np.asarray(g64), np.asarray(gmx)
    np.testing.assert_allclose(gmx, g64, rtol=1e-11, atol=1e-12 * np.abs(g64).max())


# ------------------------------------------------ the default map: claimed
@pytest.mark.parametrize("beta,nu", [(0.03, 0.5), (0.1, 0.5), (0.05, 0.8), (0.1, 1.0)])
def test_default_map_vs_oracle_grid(orc, exa, beta, nu):
    # tile 128: 13 tile columns, so that FP32 and BF16 tiles appear
    ctx = exa.Context(ts=128)
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    ref = orc.loglik(x, y, z, th)
    got = ctx.loglik(dev(x), dev(y), dev(z), th, "mixed")
    tm = ctx.timings()
    err = rel(got, ref)
    print(f"default map, 40 x 40 grid, beta={beta} nu={nu}: rel err {err:.2e} (bf16 {tm['frac_bf16']:.2f}, "
          f"fp64 {tm['frac_fp64']:.2f}, refinement steps {tm['refine_steps']:.0f})")
    assert tm["refine_steps"] == 1
    assert err <= CLAIM


@pytest.mark.parametrize("n,ts,nu", [(2000, 256, 0.8), (3000, 512, 0.5)])
def test_default_map_vs_oracle_uniform(orc, exa, n, ts, nu):
    ctx = exa.Context(ts=ts)
    x, y = inputgen.uniform(n, seed=40 + n)
    th = [1.0, 0.05, nu]
    z = orc.simulate(x, y, th, inputgen.normals(n, seed=40 + n))
    ref = orc.loglik(x, y, z, th)
    got = ctx.loglik(dev(x), dev(y), dev(z), th, "mixed")
    tm = ctx.timings()
    err = rel(got, ref)
    print(f"default map, {n} uniform points, nu={nu}: rel err {err:.2e} (bf16 {tm['frac_bf16']:.2f}, "
          f"fp64 {tm['frac_fp64']:.2f})")
    assert err <= CLAIM


def _markov_1d(n, s2, beta, gap, seed):
    t, y0 = inputgen.collinear(n, mean_gap=gap, seed=seed)
    rho = np.exp(-np.diff(t) / beta)
    e = inputgen.normals(n, seed=seed)
    z = np.empty(n)
    z[0] = math.sqrt(s2) * e[0]
    for i in range(1, n):
        z[i] = rho[i - 1] * z[i - 1] + math.sqrt(s2 * (1 - rho[i - 1] ** 2)) * e[i]
    v = s2 * (1 - rho ** 2)
    ref = -0.5 * (LN2PI + math.log(s2) + z[0] ** 2 / s2)
    ref += np.sum(-0.5 * (LN2PI + np.log(v) + (z[1:] - rho * z[:-1]) ** 2 / v))
    return t, y0, z, ref


@pytest.mark.parametrize("gap", [5e-4, 4e-3])
def test_default_map_markov_line_full_size(exa, gap):
    # nu = 1/2 on a line, n = 40,000, tile 768: the exact O(n) likelihood.
    # With mean gap 5e-4 a tile spans 3.8 beta: neighbouring tiles are FP64,
    # the next two FP32 and the rest BF16, so every precision is exercised.
    n, s2, beta = 40000, 1.0, 0.1
    t, y0, z, ref = _markov_1d(n, s2, beta, gap, seed=11)
    perm = inputgen.shuffled(n, seed=12)
    ctx = exa.Context(ts=768)
    got = ctx.loglik(dev(t[perm]), dev(y0[perm]), dev(z[perm]), [s2, beta, 0.5], "mixed")
    tm = ctx.timings()
    err = rel(got, ref)
    print(f"Markov line gap {gap}: mixed rel err vs closed form {err:.2e} (bf16 {tm['frac_bf16']:.3f}, "
          f"fp32 {tm['frac_fp32']:.3f}, fp64 {tm['frac_fp64']:.3f})")
    if gap == 5e-4:
        assert tm["frac_bf16"] > 0 and tm["frac_fp32"] > 0 and tm["frac_fp64"] > 0
    assert err <= CLAIM


@pytest.mark.parametrize("beta,nu", [(0.03, 0.5), (0.1, 0.5), (0.1, 1.0)])
def test_default_map_grid_full_size(exa, beta, nu):
    # n = 40,000 (200 x 200 jittered grid), tile 768, against the FP64 path
    x, y = inputgen.jittered_grid(200, seed=0)
    th = [1.0, beta, nu]
    ctx = exa.Context(ts=768)
    X, Y = dev(x), dev(y)
    Z = ctx.simulate(X, Y, th, dev(inputgen.normals(x.size, seed=0)))
    l64, g64 = ctx.loglik_grad(X, Y, Z, th, "fp64")
    lmx, gmx = ctx.loglik_grad(X, Y, Z, th, "mixed")
    tm = ctx.timings()
    err = rel(lmx, l64)
    gerr = np.abs(np.asarray(gmx) - np.asarray(g64)) / np.abs(np.asarray(g64)).max()
    print(f"default map, 200 x 200 grid, beta={beta} nu={nu}: rel err {err:.2e} (bf16 {tm['frac_bf16']:.2f}, "
          f"fp64 {tm['frac_fp64']:.2f}), score err / max|g| {gerr}")
    assert err <= CLAIM
    # the score is claimed at 1e-6 of max |g| where the mixed factor itself is
    # that accurate (beta = 0.03, observed 9e-9); at beta = 0.1 the factor's
    # error dominates (4e-6 at nu = 1/2, 2e-3 at nu = 1) and is recorded
    if beta == 0.03:
        assert np.all(gerr <= 1e-6)


@pytest.mark.parametrize("field", ["grid200_beta0.03", "grid150_beta0.03", "markov_line"])
def test_bf16_wide_block_same_bits(exa, field):
    # the 256 x 256 BF16 update and the 128 x 128 one form the same products
    # and sums in the same order: l and the score agree bit for bit (a ragged
    # last tile on the 150 x 150 grid: 22,500 = 29 * 768 + 228)
    if field == "markov_line":
        x, y = inputgen.collinear(40000, 5e-4, seed=0)
        th = [1.0, 0.1, 0.5]
    else:
        m = 200 if field.startswith("grid200") else 150
        x, y = inputgen.jittered_grid(m, seed=0)
        th = [1.0, 0.03, 0.5]
    ctx = exa.Context(ts=768)
    X, Y = dev(x), dev(y)
    Z = ctx.simulate(X, Y, th, dev(inputgen.normals(x.size, seed=0)))
    wide = ctx.loglik_grad(X, Y, Z, th, "mixed")
    tm = ctx.timings()
    ctx.set_mixed_bf16_block(128)
    narrow = ctx.loglik_grad(X, Y, Z, th, "mixed")
    print(f"{field}: bf16 {tm['frac_bf16']:.2f}, l {wide[0]!r} vs {narrow[0]!r}")
    assert tm["frac_bf16"] > 0.1
    assert wide == narrow


def test_refinement_steps_lower_the_error(exa):
    # 200 x 200 grid, beta = 0.1, nu = 1/2: the plain mixed solve, one and two
    # refinement steps; each step may only be taken if its residual shrinks
    x, y = inputgen.jittered_grid(200, seed=0)
    th = [1.0, 0.1, 0.5]
    ctx = exa.Context(ts=768)
    X, Y = dev(x), dev(y)
    Z = ctx.simulate(X, Y, th, dev(inputgen.normals(x.size, seed=0)))
    l64 = ctx.loglik(X, Y, Z, th, "fp64")
    errs = []
    for steps in (0, 1, 2):
        ctx.set_mixed_refinement(steps)
        errs.append(rel(ctx.loglik(X, Y, Z, th, "mixed"), l64))
    print(f"refinement steps 0, 1, 2: rel err {errs}")
    assert errs[1] < errs[0] and errs[2] <= errs[1] * 1.5


# ---------------------------------- maps that make no claim: the record
def test_unclaimed_maps_record_errors(orc, exa):
    x, y = inputgen.jittered_grid(40, seed=2)
    rows = []
    for beta, nu in ((0.03, 0.5), (0.1, 0.5), (0.1, 1.0)):
        th = [1.0, beta, nu]
        z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
        ref = orc.loglik(x, y, z, th)
        fr = {}
        for label, band, fb in (("fp32 only", 0.0, 0.0), ("bf16 beyond 3 beta", 3.0, 0.0),
                                ("bf16 beyond 6 beta", 6.0, 0.0), ("fp32 + fp64 band 0.5 beta", 0.0, 0.5)):
            ctx = exa.Context(ts=256, band_factor=band, fp64_band=fb)
            ctx.set_mixed_refinement(0)
            st, got, info = ctx.loglik_status(dev(x), dev(y), dev(z), th, "mixed")
            tm = ctx.timings()
            assert st in (exa.OK, exa.ENOTPD)
            fr[label] = tm["frac_bf16"]
            rows.append(f"beta={beta} nu={nu} {label}: "
                        + (f"rel err {rel(got, ref):.2e}" if st == exa.OK else f"ENOTPD at {info}")
                        + f" (bf16 {tm['frac_bf16']:.2f}, fp64 {tm['frac_fp64']:.2f})")
        # structure: a wider BF16 band keeps more tiles out of BF16, none at 0
        assert fr["fp32 only"] == 0.0 and fr["bf16 beyond 6 beta"] <= fr["bf16 beyond 3 beta"]
    # the default map outside the claimed range: a smoother, longer-range field
    th = [1.0, 0.2, 1.5]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    ref = orc.loglik(x, y, z, th)
    ctx = exa.Context(ts=128)
    st, got, info = ctx.loglik_status(dev(x), dev(y), dev(z), th, "mixed")
    assert st in (exa.OK, exa.ENOTPD)
    tm = ctx.timings()
    rows.append(f"default map, beta=0.2 nu=1.5 (outside the claimed range), tile 128: "
                + (f"rel err {rel(got, ref):.2e}" if st == exa.OK else f"ENOTPD at {info}")
                + f" (bf16 {tm['frac_bf16']:.2f}, fp64 {tm['frac_fp64']:.2f})")
    print("\n".join(rows))


@pytest.mark.parametrize("beta,nu", [(0.1, 0.5), (0.1, 1.0)])
def test_distance_fp64_band_reduces_error(orc, exa, beta, nu):
    # 60 x 60 grid, ts 128: NT = 29, 406 off-diagonal tiles; the pool holds up
    # to half of them, the closest first
    x, y = inputgen.jittered_grid(60, seed=6)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=6))
    ref = orc.loglik(x, y, z, th)
    X, Y, Z = dev(x), dev(y), dev(z)
    errs = {}
    for fb in (0.0, 0.5):
        ctx = exa.Context(ts=128, band_factor=0.0, fp64_band=fb)
        ctx.set_mixed_refinement(0)
        st, got, _ = ctx.loglik_status(X, Y, Z, th, "mixed")
        errs[fb] = (abs(got - ref) / abs(ref) if st == exa.OK else math.inf, ctx.timings()["frac_fp64"])
    print(f"beta={beta} nu={nu}: " + ", ".join(f"fp64 band {b}: rel {e:.2e} (fp64 tiles {f:.2f})"
                                               for b, (e, f) in errs.items()))
    assert errs[0.0][1] == 0.0 and 0.0 < errs[0.5][1] <= 203 / 406 + 1e-12
    assert errs[0.5][0] < errs[0.0][0]


# ------------------------------------------------------------ statuses
def test_mixed_notpd_status(exa):
    ctx = exa.Context(ts=128)
    st, ll, info = ctx.loglik_status(dev([0.3, 0.3]), dev([0.2, 0.2]), dev([1.0, 0.5]), [4.0, 0.1, 0.5], "mixed")
    assert st == exa.ENOTPD and ll == -math.inf and info in (1, 2)


@pytest.mark.parametrize("band", [3.0, 1.0])
def test_mixed_failure_is_reported_not_a_number(orc, exa, band):
    # BF16 close to the diagonal of a smooth field can push the smallest
    # eigenvalue below zero: then the status is ENOTPD with l = -inf and a
    # valid caller index, never a finite wrong value; an OK status must come
    # with a finite l
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, 0.1, 1.0]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    ctx = exa.Context(ts=256, band_factor=band)
    ctx.set_mixed_refinement(0)
    st, ll, info = ctx.loglik_status(dev(x), dev(y), dev(z), th, "mixed")
    print(f"bf16 beyond {band} beta, smooth field: status {st}, l {ll}, info {info}")
    if st == exa.OK:
        assert math.isfinite(ll) and info == 0
    else:
        assert st == exa.ENOTPD and ll == -math.inf and 1 <= info <= x.size


# ------------------------------------------------------------ score
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


@pytest.mark.parametrize("beta,nu", [(0.03, 0.5), (0.1, 0.5), (0.1, 1.0)])
def test_mixed_score_record(orc, exa, beta, nu):
    # the a^T dSigma a term uses the refined a, the trace term the mixed
    # inverse factor (FP64 on the factor's FP64 band, FP32 elsewhere).  The
    # default map claims 1e-8 of max |g| against the oracle here (observed
    # <= 4e-10); the FP32-only map is printed as a record.
    x, y = inputgen.jittered_grid(40, seed=2)
    th = [1.0, beta, nu]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=2))
    lref, gref = orc.loglik_grad(x, y, z, th)
    gref = np.asarray(gref)
    for label, ctx in (("default map", exa.Context(ts=256)), ("fp32 only", exa.Context(ts=256, band_factor=0.0))):
        if label == "fp32 only":
            ctx.set_mixed_refinement(0)
        lmx, gmx = ctx.loglik_grad(dev(x), dev(y), dev(z), th, "mixed")
        err = np.abs(np.asarray(gmx) - gref)
        print(f"mixed score beta={beta} nu={nu} {label}: l rel {rel(lmx, lref):.2e}, score err / max|g| = "
              f"{err / np.abs(gref).max()}, per component {err / np.abs(gref)}")
        assert np.all(np.isfinite(gmx))
        if label == "default map":
            assert np.all(err <= 1e-8 * np.abs(gref).max())


def test_mixed_lbfgsb_mle_matches_fp64(orc, exa):
    ctx = exa.Context(ts=256)
    x, y = inputgen.jittered_grid(30, seed=4)
    th = [1.0, 0.1, 0.5]
    z = orc.simulate(x, y, th, inputgen.normals(x.size, seed=4))
    X, Y, Z = dev(x), dev(y), dev(z)
    lb, ub, t0 = [0.01, 0.01, 0.1], [5.0, 2.0, 2.0], [0.5, 0.3, 0.5]
    th64, l64, s64 = ctx.mle(X, Y, Z, lb, ub, theta0=t0, tol=1e-7, method="lbfgsb", precision="fp64")
    thmx, lmx, smx = ctx.mle(X, Y, Z, lb, ub, theta0=t0, tol=1e-7, method="lbfgsb", precision="mixed")
    l64_at_mx = ctx.loglik(X, Y, Z, thmx, "fp64")
    print("fp64", th64, l64, s64, "mixed", thmx, lmx, smx, "fp64 l at the mixed estimate", l64_at_mx)
    assert smx["n_grad_evals"] > 0
    assert abs(l64_at_mx - l64) <= CLAIM * abs(l64)


def test_mle_mixed_search_with_fp64_finish(exa):
    # 48 x 48 jittered grid, theta = (1, 0.1, 0.5): the mixed-precision search
    # followed by an FP64 finish reaches the FP64 L-BFGS-B optimum to 1e-6 of l
    x, y = inputgen.jittered_grid(48, seed=4)
    n = x.size
    ctx = exa.Context(ts=256)
    th_true = [1.0, 0.1, 0.5]
    e = torch.as_tensor(inputgen.normals(n, seed=4), device="cuda")
    X, Y = dev(x), dev(y)
    Z = ctx.simulate(X, Y, th_true, e)
    lb, ub, th0 = [0.01, 0.01, 0.1], [5.0, 2.0, 3.0], [0.5, 0.3, 0.5]
    th64, ll64, st64 = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-7, method="lbfgsb", precision="fp64")
    thm, llm, stm = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-7, method="lbfgsb_fp64_finish",
                            precision="mixed")
    print(f"fp64 {th64} {ll64} {st64}\nmixed+finish {thm} {llm} {stm}")
    assert st64["status"] == "OK" and stm["status"] == "OK"
    assert 0 < stm["n_fp64_finish_evals"] < stm["n_grad_evals"]
    # the reported value is an FP64 likelihood at the returned point
    assert ctx.loglik(X, Y, Z, thm) == llm
    assert abs(llm - ll64) <= CLAIM * abs(ll64)
