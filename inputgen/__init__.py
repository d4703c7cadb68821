"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method: it only draws locations and
standard-normal vectors with numpy's PCG64 (``default_rng(seed)``).  The field
values z = L e that need a Cholesky factor are produced by the caller (the
oracle in tests, the library's simulator in the benchmark).

Location recipes (the paper's simulation studies use U[0,1]^2 locations,
Section 3 Example 1, and regular grids; "m x m jittered grid" follows the
reading documented with the benchmark):
  * ``jittered_grid(m)``: centres (i + 0.5)/m, i = 0..m-1, each coordinate
    moved by U(-0.4, 0.4)/m, so points stay in [0,1]^2 and no two are closer
    than 0.2/m;
  * ``uniform(n)``: U[0,1]^2;
  * ``collinear(n, spacing)``: sorted points on the x axis with random gaps,
    for the one-dimensional Markov (Ornstein-Uhlenbeck) pin at nu = 1/2;
  * ``clusters(...)``: well separated square clusters, for the
    block-additivity pin.
"""
from __future__ import annotations

import numpy as np


def jittered_grid(m: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    c = (np.arange(m) + 0.5) / m
    gx, gy = np.meshgrid(c, c, indexing="ij")
    x = gx.ravel() + rng.uniform(-0.4, 0.4, m * m) / m
    y = gy.ravel() + rng.uniform(-0.4, 0.4, m * m) / m
    return x.astype(np.float64), y.astype(np.float64)


def uniform(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = rng.random(n)
    return x, y


def normals(n: int, seed: int = 0):
    rng = np.random.default_rng(seed + 7919)
    return rng.standard_normal(n)


def smooth_field(x, y, seed: int = 0):
    """Observations that vary smoothly over the locations: a sum of 16 plane
    waves cos(2 pi (kx x + ky y) + phase), kx, ky = 0..3, with N(0, 1)
    amplitudes and U(0, 2 pi) phases (numpy PCG64, seed).  Used where a
    check needs z^T Sigma^-1 z to be insensitive to rounding (a white-noise z
    weights Sigma's smallest eigenvalues)."""
    rng = np.random.default_rng(seed + 104729)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.zeros_like(x)
    for kx in range(4):
        for ky in range(4):
            a, ph = rng.standard_normal(), rng.uniform(0.0, 2.0 * np.pi)
            z += a * np.cos(2.0 * np.pi * (kx * x + ky * y) + ph)
    return z


def collinear(n: int, mean_gap: float, seed: int = 0):
    """Sorted 1-D locations on y = 0 with gaps U(0.5, 1.5) * mean_gap."""
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(0.5, 1.5, n) * mean_gap
    t = np.cumsum(gaps)
    return t.astype(np.float64), np.zeros(n)


def clusters(n_per: int, n_clusters: int, width: float, separation: float, seed: int = 0):
    """n_clusters square clusters of side ``width`` on a line, ``separation`` apart.

    Returns x, y and the cluster label of each point; points of a cluster
    are contiguous, clusters are given in a shuffled order so that the
    caller cannot rely on any ordering.
    """
    rng = np.random.default_rng(seed)
    xs, ys, lab = [], [], []
    for c in range(n_clusters):
        xs.append(c * separation + rng.random(n_per) * width)
        ys.append(rng.random(n_per) * width)
        lab.append(np.full(n_per, c))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    lab = np.concatenate(lab)
    perm = rng.permutation(x.size)
    return x[perm], y[perm], lab[perm]


def shuffled(n: int, seed: int = 0):
    return np.random.default_rng(seed + 104729).permutation(n)


def corner_clusters(n_per: int, width: float, separation: float, seed: int = 0):
    """Four square clusters of side ``width`` at the corners of a square of
    side ``separation``; labels 0..3, points shuffled."""
    rng = np.random.default_rng(seed)
    xs, ys, lab = [], [], []
    for c, (cx, cy) in enumerate([(0.0, 0.0), (separation, 0.0), (0.0, separation), (separation, separation)]):
        xs.append(cx + rng.random(n_per) * width)
        ys.append(cy + rng.random(n_per) * width)
        lab.append(np.full(n_per, c))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    lab = np.concatenate(lab)
    perm = rng.permutation(x.size)
    return x[perm], y[perm], lab[perm]
