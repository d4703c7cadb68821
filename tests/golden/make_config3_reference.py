"""Reference l(theta) for the n = 40,000 FP64 workload, written by the oracle's
covariance (eq. (3) with its own K_nu) factored by LAPACK (torch's CPU
LAPACK) as a library step.

Workload: 40,000 locations U[0,1]^2 (inputgen.uniform(40000, seed=0)),
theta = (sigma^2, beta, nu) = (1, 0.1, 1.0), z = inputgen.normals(40000,
seed=0) (standard normal; a parity check needs the same z on both sides, not a
draw from the model).  Writes config3_loglik.json: l of eq. (2), log det Sigma
(twice the sum of the log pivots) and z^T Sigma^-1 z = |L^-1 z|^2.

Run on the CPU (about 26 GB for Sigma and its factor; minutes with OpenMP and
a threaded LAPACK):  python tests/golden/make_config3_reference.py [threads]
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import inputgen  # noqa: E402
import oracle  # noqa: E402


def main() -> int:
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    oracle.set_threads(threads)
    n, theta = 40000, [1.0, 0.1, 1.0]
    x, y = inputgen.uniform(n, seed=0)
    z = inputgen.smooth_field(x, y, seed=0)
    t0 = time.time()
    S = oracle.matern_cov(x, y, theta)
    t1 = time.time()
    torch.set_num_threads(threads)
    L = torch.linalg.cholesky(torch.from_numpy(S))
    del S
    t2 = time.time()
    logdet = 2.0 * float(torch.log(torch.diagonal(L)).sum())
    v = torch.linalg.solve_triangular(L, torch.from_numpy(z)[:, None], upper=False)
    q = float((v * v).sum())
    ll = -0.5 * (n * np.log(2.0 * np.pi) + logdet + q)
    out = {
        "workload": "n = 40,000 U[0,1]^2 (inputgen.uniform(40000, seed=0)), theta = (1, 0.1, 1.0), "
                    "z = inputgen.smooth_field(x, y, seed=0)",
        "reference": "oracle covariance (eq. (3), own K_nu), LAPACK Cholesky, eq. (2)",
        "n": n, "theta": theta, "loglik": ll, "logdet": logdet, "quad_form": q,
        "seconds": {"covariance": t1 - t0, "cholesky": t2 - t1}, "threads": threads,
    }
    with open(os.path.join(HERE, "config3_loglik.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
