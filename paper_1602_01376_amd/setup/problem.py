"""Seeded problem generator: points, tree, skeletons and P for each workload.

A `Problem` holds everything both the GPU path and its checker consume, all
in tree order.  Workloads (sizes and value structure; the paper's datasets
are not available, so these are synthetic stand-ins):

  tiny     N=4,096  d=8   4 unit Gaussians, m=128 (L=5), s=64, h=1.0,  lambda=1e-2
  covtype  N=65,536 d=54  8 Gaussians with per-dim scales in [0.5,2], m=256
           (L=8), s=128, h=2.0, lambda=1e-3, 16 RHS
  susy     N=1,048,576 d=8 16 unit Gaussians, L=12, uneven leaves 64..512,
           adaptive s in [32,256] at tau=1e-5, h=0.5, lambda=1e-4, 1 or 64 RHS
  susy-wide  the susy points and tree with h=1.0, tau=1e-13, lambda=1e-2:
           ranks spread over 32..256 (median about 50, top levels above 200)
  mnist    N=262,144 d=784 sparse [0,1] coordinates stored fp32, m=512 (L=9),
           s=256, h=4.0, lambda=1e-2
  normal   N=4,194,304 d=64 32 unit Gaussians, m=512 (L=13), s=256, h=1.5,
           lambda sweep logspace(-6,-1,8), 32 RHS

Seeds: data 1000+i, setup 2000+i, rhs 3000+i for workload number i (1..5).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import balltree, points, skeleton


@dataclasses.dataclass
class Problem:
    X: np.ndarray            # (N, d) tree-ordered points, float64 (float32 for mnist)
    perm: np.ndarray         # perm[t] = original row of tree position t
    depth: int               # L; leaves at level L, root at level 0
    leaf_offsets: np.ndarray  # int64 [2^L + 1]
    skel_offsets: np.ndarray  # int64 [n_nodes + 1], heap node order
    skel_index: np.ndarray    # int32 tree-order point ids
    p_offsets: np.ndarray     # int64 [n_nodes + 1]
    p_values: np.ndarray      # float64, leaf s x m / internal s x (s_l+s_r), row-major
    h: float
    name: str = ""
    lam: float = 0.0          # default regularization of the workload
    nrhs: int = 1

    # --- pure indexing helpers (no arithmetic of the method) ---
    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_nodes(self) -> int:
        return (1 << (self.depth + 1)) - 1

    def level_of(self, node: int) -> int:
        return int(math.floor(math.log2(node + 1)))

    def node_range(self, node: int):
        k = self.level_of(node)
        j = node - ((1 << k) - 1)
        span = 1 << (self.depth - k)
        return int(self.leaf_offsets[j * span]), int(self.leaf_offsets[(j + 1) * span])

    def is_leaf(self, node: int) -> bool:
        return self.level_of(node) == self.depth

    def skel(self, node: int) -> np.ndarray:
        return self.skel_index[self.skel_offsets[node]:self.skel_offsets[node + 1]]

    def s(self, node: int) -> int:
        return int(self.skel_offsets[node + 1] - self.skel_offsets[node])

    def P(self, node: int) -> np.ndarray:
        """Stored interpolation matrix of `node` as an (s, cols) view."""
        a, b = self.p_offsets[node], self.p_offsets[node + 1]
        s = self.s(node)
        if s == 0:
            return np.zeros((0, 0))
        return self.p_values[a:b].reshape(s, -1)

    def astuple(self):
        return dataclasses.astuple(self)


WORKLOADS = {
    "tiny": dict(idx=1, n=4096, d=8, mixture=4, scale_range=None, depth=5,
                 split="median", s_fixed=64, n_samp=256, h=1.0, lam=1e-2, nrhs=1),
    "covtype": dict(idx=2, n=65536, d=54, mixture=8, scale_range=(0.5, 2.0), depth=8,
                    split="median", s_fixed=128, n_samp=256, h=2.0, lam=1e-3, nrhs=16),
    "susy": dict(idx=3, n=1 << 20, d=8, mixture=16, scale_range=None, depth=12,
                 split="random", leaf_min=64, leaf_max=512, s_min=32, s_max=256,
                 tau=1e-5, n_samp=320, h=0.5, lam=1e-4, nrhs=1),
    # the same points and tree as susy with a smoother kernel and a tighter
    # ID tolerance, so that the adaptive ranks spread over 32..256
    "susy-wide": dict(idx=3, n=1 << 20, d=8, mixture=16, scale_range=None, depth=12,
                      split="random", leaf_min=64, leaf_max=512, s_min=32, s_max=256,
                      tau=1e-13, n_samp=320, h=1.0, lam=1e-2, nrhs=1),
    "mnist": dict(idx=4, n=1 << 18, d=784, sparse=True, depth=9, split="median",
                  s_fixed=256, n_samp=320, h=4.0, lam=1e-2, nrhs=1),
    "normal": dict(idx=5, n=1 << 22, d=64, mixture=32, scale_range=None, depth=13,
                   split="median", s_fixed=256, n_samp=320, h=1.5, lam=1e-1, nrhs=32),
}


def make_problem(workload: str = "tiny", *, n: int | None = None, depth: int | None = None,
                 full_skeletons: bool = False, s_fixed: int | None = None,
                 h: float | None = None, workers=None, progress=None, **overrides) -> Problem:
    """Generate a seeded problem.

    `n`/`depth` scale a workload down while keeping its structure (leaf size
    bounds, rank rule, value distribution).  `full_skeletons=True` makes
    every node's skeleton its full candidate set (P a permutation), which
    turns K~ into K exactly.  `progress(text)`, if given, reports each step.
    """
    cfg = dict(WORKLOADS[workload])
    cfg.update(overrides)
    if n is not None:
        cfg["n"] = n
    if depth is not None:
        cfg["depth"] = depth
    if s_fixed is not None:
        cfg["s_fixed"] = s_fixed
    if h is not None:
        cfg["h"] = h
    i = cfg["idx"]
    N, d, L = cfg["n"], cfg["d"], cfg["depth"]
    if cfg.get("sparse"):
        X = points.sparse_unit_cube(N, d, seed=1000 + i)
    else:
        X = points.gaussian_mixture(N, d, cfg["mixture"], seed=1000 + i,
                                    scale_range=cfg.get("scale_range"))
    perm, leaf_offsets = balltree.build_tree(
        X, L, split=cfg["split"], leaf_min=cfg.get("leaf_min", 0),
        leaf_max=cfg.get("leaf_max", 0), seed=2000 + i)
    X = np.ascontiguousarray(X[perm])
    if progress is not None:
        progress(f"points and ball tree done (N={N}, d={d}, depth {L})")
    if "s_fixed" in cfg and cfg["s_fixed"] is not None:
        rank = dict(s_fixed=cfg["s_fixed"])
    else:
        rank = dict(s_min=cfg["s_min"], s_max=cfg["s_max"], tau=cfg["tau"])
    so, si, po, pv = skeleton.skeletonize(
        X, L, leaf_offsets, cfg["h"], n_samp=cfg["n_samp"], seed=2000 + i,
        full=full_skeletons, workers=workers, progress=progress, **rank)
    return Problem(X=X, perm=perm, depth=L, leaf_offsets=leaf_offsets,
                   skel_offsets=so, skel_index=si, p_offsets=po, p_values=pv,
                   h=float(cfg["h"]), name=workload, lam=float(cfg["lam"]),
                   nrhs=int(cfg["nrhs"]))


def rhs_for(problem: Problem, nrhs: int | None = None, seed: int | None = None) -> np.ndarray:
    """Seeded right-hand sides for a problem, (N, nrhs) float64 Fortran order."""
    idx = WORKLOADS[problem.name]["idx"] if problem.name in WORKLOADS else 0
    return points.random_rhs(problem.n, nrhs or problem.nrhs,
                             seed=3000 + idx if seed is None else seed)
