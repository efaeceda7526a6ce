"""Seeded synthetic point sets that stand in for the paper's datasets.

The paper's experiments use COVTYPE, SUSY, MNIST and a NORMAL point cloud
(Section IV, dataset table).  None of those are available here, so every
workload is a seeded synthetic set with the dimension and value structure of
one of them.  Nothing in this module evaluates a kernel or touches the
factorization: it only draws numbers.
"""
from __future__ import annotations

import numpy as np


def gaussian_mixture(n: int, d: int, n_components: int, seed: int,
                     center_range: float = 5.0, scale_range=None) -> np.ndarray:
    """n points from an equal-weight mixture of `n_components` Gaussians.

    Centres are uniform in [-center_range, center_range]^d.  With
    `scale_range=None` every component has unit variance; otherwise each
    component draws a per-dimension standard deviation uniform in
    `scale_range`.  Component counts are equal (up to one point) and the
    rows are shuffled.  Returns an (n, d) float64 array.
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-center_range, center_range, size=(n_components, d))
    if scale_range is None:
        scales = np.ones((n_components, d))
    else:
        scales = rng.uniform(scale_range[0], scale_range[1], size=(n_components, d))
    counts = np.full(n_components, n // n_components, dtype=np.int64)
    counts[: n - counts.sum()] += 1
    labels = np.repeat(np.arange(n_components), counts)
    rng.shuffle(labels)
    z = rng.standard_normal((n, d))
    return centers[labels] + z * scales[labels]


def sparse_unit_cube(n: int, d: int, seed: int, p_zero: float = 0.9) -> np.ndarray:
    """Sparse-image-like points: each coordinate is 0 with probability
    `p_zero`, otherwise uniform in [0, 1].  Returned as float32, the storage
    precision of this workload."""
    rng = np.random.default_rng(seed)
    vals = rng.uniform(0.0, 1.0, size=(n, d)).astype(np.float32)
    mask = rng.uniform(0.0, 1.0, size=(n, d)) < p_zero
    vals[mask] = 0.0
    return vals


def low_intrinsic_normal(n: int, d: int, seed: int, intrinsic: int = 6,
                         noise: float = 0.05) -> np.ndarray:
    """A normal cloud of intrinsic dimension `intrinsic` embedded in d
    dimensions by a random orthonormal map, plus isotropic noise: the recipe
    the paper describes for its NORMAL weak-scaling data (Section IV,
    datasets paragraph)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, intrinsic))
    q, _ = np.linalg.qr(rng.standard_normal((d, intrinsic)))
    return z @ q.T + noise * rng.standard_normal((n, d))


def random_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides b ~ N(0, 1), shape (n, nrhs), float64, column-major
    in memory (Fortran order) so each column is contiguous."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, nrhs)))
