"""Complete binary ball tree used to order the points (Section II-A/II-B).

The paper partitions the points with a balanced binary ball tree and orders
the rows and columns of K by it, so that every tree node owns a contiguous
index range.  It names the tree type but not the split rule.  The rule used
here: project the node's points on the line through two far-apart points
(p1 = farthest from the centroid, p2 = farthest from p1) and split the sorted
projections either at the median or at a clamped random quantile (the
uneven-leaf workload).  Every leaf sits at depth L, so node (level k, index j)
owns leaves [j*2^(L-k), (j+1)*2^(L-k)).
"""
from __future__ import annotations

import numpy as np


def _split_direction(pts: np.ndarray) -> np.ndarray:
    c = pts.mean(axis=0)
    p1 = pts[np.argmax(((pts - c) ** 2).sum(axis=1))]
    p2 = pts[np.argmax(((pts - p1) ** 2).sum(axis=1))]
    v = p2 - p1
    if not np.any(v):
        v = np.zeros(pts.shape[1])
        v[0] = 1.0
    return v


def build_tree(X: np.ndarray, depth: int, split: str = "median",
               leaf_min: int = 0, leaf_max: int = 0, quantile=(0.3, 0.7),
               seed: int = 0):
    """Order the points of X by a complete ball tree of the given depth.

    Returns (perm, leaf_offsets): `perm[t]` is the original row of the point
    at tree position t; `leaf_offsets` (2^depth + 1 int64) bounds each leaf.

    split="median": children get floor/ceil halves.
    split="random": the left child gets a quantile q ~ U[quantile] of the
    points, clamped so that every leaf below can stay within
    [leaf_min, leaf_max].
    """
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = np.arange(n, dtype=np.int64)
    bounds = [0, n]
    for k in range(depth):
        sub_leaves = 1 << (depth - k - 1)  # leaves under each child
        new_bounds = [0]
        for j in range(1 << k):
            lo, hi = bounds[j], bounds[j + 1]
            cnt = hi - lo
            idx = perm[lo:hi]
            pts = X[idx].astype(np.float64)
            proj = pts @ _split_direction(pts)
            order = np.argsort(proj, kind="stable")
            if split == "median":
                nl = cnt // 2
            elif split == "random":
                q = rng.uniform(quantile[0], quantile[1])
                nl = int(round(q * cnt))
                a = max(leaf_min * sub_leaves, cnt - leaf_max * sub_leaves)
                b = min(leaf_max * sub_leaves, cnt - leaf_min * sub_leaves)
                if a > b:
                    raise ValueError("leaf size bounds cannot be met")
                nl = min(max(nl, a), b)
            else:
                raise ValueError(f"unknown split rule {split!r}")
            perm[lo:hi] = idx[order]
            new_bounds.append(lo + nl)
            new_bounds.append(hi)
        bounds = new_bounds
    return perm, np.asarray(bounds, dtype=np.int64)
