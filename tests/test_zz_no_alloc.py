"""The allocation-free entry point (exageo_loglik_grad_noalloc, the library's
fixed device scratch) against exageo_loglik_grad on the same inputs, through
the C ABI: two calls in a row, the second with a smaller problem, so the
second runs on scratch that still holds the first call's contents."""
import numpy as np
import pytest

import inputgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def test_noalloc_matches_loglik_grad_two_calls(orc):
    import paper_1908_06936_amd as exa

    ctx = exa.Context(ts=256)
    th = [1.0, 0.1, 0.8]
    for n, seed in ((3900, 61), (1100, 62)):
        print(f"noalloc case n={n} seed={seed}", flush=True)
        x, y = inputgen.uniform(n, seed=seed)
        X, Y = dev(x), dev(y)
        Z = ctx.simulate(X, Y, th, dev(inputgen.normals(n, seed=seed)))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        st, ll_na, g_na, info = ctx.loglik_grad_noalloc(X, Y, Z, th)
        st1, l1_na, g1, _ = ctx.loglik_grad_noalloc(X, Y, Z, th, with_grad=False)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before  # the binding took no torch memory either
        assert st == exa.OK and info == 0, ctx.last_error()
        assert st1 == exa.OK and g1 is None
        ll, g = ctx.loglik_grad(X, Y, Z, th)
        print(f"n={n}: noalloc l={ll_na!r} g={g_na}; loglik_grad l={ll!r} g={g}; "
              f"bitwise equal: {ll_na == ll and g_na == g}")
        assert ll_na == pytest.approx(ll, rel=1e-12)
        assert l1_na == pytest.approx(ll, rel=1e-12)
        np.testing.assert_allclose(g_na, g, rtol=1e-10, atol=1e-10 * max(abs(v) for v in g))
        if n <= 1500:
            ll_o, g_o = orc.loglik_grad(x, y, Z.cpu().numpy(), th)
            assert ll_na == pytest.approx(ll_o, rel=1e-10)
            np.testing.assert_allclose(g_na, g_o, rtol=1e-8, atol=1e-8 * np.abs(g_o).max())


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import paper_1908_06936_amd as exa

    ctx = exa.Context(ts=256)
    n = 20000
    x, y = inputgen.uniform(n, seed=63)
    st, ll, g, info = ctx.loglik_grad_noalloc(dev(x), dev(y), dev(inputgen.normals(n, seed=63)), [1.0, 0.1, 0.5])
    assert st == exa.ENOMEM
    assert "fixed scratch" in ctx.last_error()
