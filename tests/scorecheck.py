"""Per-component comparison of a score vector (dl/dtheta) with a reference.

Each component g_k = 1/2 a^T dSigma_k a - 1/2 tr(Sigma^-1 dSigma_k) is the
difference of two sums of size about n / (2 theta_k) (for sigma^2 exactly
q / (2 sigma^4) and n / (2 sigma^2)), so its FP64 rounding scales with
n / theta_k, not with |g_k|: the bound is rtol |g_ref,k| plus 1e-11 n / theta_k,
which only matters for a component near zero.  No component is judged by the
size of the others.
"""
import numpy as np


def assert_score_close(g, g_ref, n, theta, rtol=1e-8, floor=1e-11):
    g = np.asarray(g, dtype=np.float64)
    g_ref = np.asarray(g_ref, dtype=np.float64)
    th = np.asarray(theta, dtype=np.float64)
    bound = rtol * np.abs(g_ref) + floor * n / th
    err = np.abs(g - g_ref)
    print(f"score per component: rel err {err / np.maximum(np.abs(g_ref), 1e-300)}, bound {bound}")
    assert np.all(err <= bound), f"score {g} vs reference {g_ref}: errors {err} above {bound}"
