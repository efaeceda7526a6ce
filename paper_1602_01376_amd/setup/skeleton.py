"""ASKIT skeletonization: skeleton sets and interpolation matrices P.

This is the upstream ASKIT step (Section II-B), not part of the INV-ASKIT
factorization: its outputs (skeleton ids and P) are inputs of both the
factorization and its checker.  For every non-root node c the candidate
columns are c's own points (leaf) or the union of the children's skeletons
[l~ | r~] (internal node, nested skeletons).  Rows are sampled uniformly from
points outside c; the skeleton is the pivot prefix of a column-pivoted QR of
the sampled block, and P comes from the interpolative decomposition
P[:, piv] = [I | R11^-1 R12].  The paper samples rows through nearest
neighbours and leaves the rank rule at "below a tolerance"; the reading here
is uniform sampling and rank = #{k : |R_kk| >= tau |R_11|}, clamped.

Leaf P is s x |c| with columns in the leaf's tree order; internal P is
s x (s_l + s_r) with columns [l~ | r~].  Both are stored row-major.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np
import scipy.linalg as sla


def _sample_kernel(XA: np.ndarray, XB: np.ndarray, h: float) -> np.ndarray:
    """Gaussian kernel block used only to choose skeletons (accuracy of this
    block affects how well K~ approximates K, not the solver it feeds)."""
    A = XA.astype(np.float64)
    B = XB.astype(np.float64)
    d2 = (A * A).sum(1)[:, None] + (B * B).sum(1)[None, :] - 2.0 * (A @ B.T)
    np.maximum(d2, 0.0, out=d2)
    return np.exp(-0.5 * d2 / (h * h))


def _interp_decomp(Kmat: np.ndarray, rank_rule):
    """Column-pivoted QR based interpolative decomposition of Kmat.
    Returns (pivot order, rank s, T) with Kmat[:, piv[s:]] ~= Kmat[:, piv[:s]] @ T."""
    R, piv = sla.qr(Kmat, mode="r", pivoting=True, check_finite=False)
    ncol = Kmat.shape[1]
    kmax = min(R.shape[0], ncol)
    diag = np.abs(np.diag(R[:kmax, :kmax]))
    s = rank_rule(diag)
    s = max(1, min(s, kmax))
    R11 = R[:s, :s]
    R12 = R[:s, s:]
    if s == ncol:
        return piv, s, np.zeros((s, 0))
    tiny = diag[0] * 1e-12 if diag[0] > 0 else 0.0
    if diag[0] > 0 and np.min(np.abs(np.diag(R11))) > tiny:
        T = sla.solve_triangular(R11, R12, check_finite=False)
    else:
        T = np.linalg.lstsq(R11, R12, rcond=1e-12)[0]
    if not np.all(np.isfinite(T)):
        T = np.linalg.lstsq(R11, R12, rcond=1e-12)[0]
    return piv, s, T


def _node_skeleton(node, cand, lo, hi, X, h, n_samp, rank_rule, seed, full):
    n = X.shape[0]
    ncand = cand.shape[0]
    rng = np.random.default_rng([seed, node])
    if full:
        # Every candidate is a skeleton, in a random order: P is then a
        # permutation and K~ equals K exactly.
        order = rng.permutation(ncand)
        skel = cand[order]
        P = np.zeros((ncand, ncand))
        P[np.arange(ncand), order] = 1.0
        return skel, P
    outside = n - (hi - lo)
    ns = min(n_samp, outside)
    samp = rng.choice(outside, size=ns, replace=False)
    samp = np.where(samp >= lo, samp + (hi - lo), samp)
    Kmat = _sample_kernel(X[samp], X[cand], h)
    piv, s, T = _interp_decomp(Kmat, rank_rule)
    P = np.zeros((s, ncand))
    P[np.arange(s), piv[:s]] = 1.0
    P[:, piv[s:]] = T
    skel = cand[piv[:s]]
    return skel, P


def skeletonize(X, depth, leaf_offsets, h, *, s_fixed=None, s_min=1, s_max=None,
                tau=None, n_samp=256, seed=0, full=False, workers=None, progress=None):
    """Build skeletons and P for every non-root node, bottom-up.

    `progress(text)`, if given, is called after each level.

    Returns (skel_offsets, skel_index, p_offsets, p_values) in heap node
    order (root = 0, children of i are 2i+1 and 2i+2).  The root has no
    skeleton and no P (it has no sibling).
    """
    L = depth
    n_nodes = (1 << (L + 1)) - 1
    skel = [None] * n_nodes
    pmat = [None] * n_nodes

    if s_fixed is not None:
        def rank_rule(diag):
            return int(s_fixed)
    else:
        def rank_rule(diag):
            if diag[0] == 0:
                return s_min
            s = int(np.count_nonzero(diag >= tau * diag[0]))
            return int(min(max(s, s_min), s_max))

    if workers is None:
        workers = min(16, os.cpu_count() or 1)

    def run_level(jobs):
        if workers <= 1 or len(jobs) < 8:
            return [_node_skeleton(*j) for j in jobs]
        try:
            from threadpoolctl import threadpool_limits
        except ImportError:  # pragma: no cover
            threadpool_limits = None
        def work(j):
            return _node_skeleton(*j)
        if threadpool_limits is not None:
            with threadpool_limits(1):
                with cf.ThreadPoolExecutor(workers) as ex:
                    return list(ex.map(work, jobs))
        with cf.ThreadPoolExecutor(workers) as ex:
            return list(ex.map(work, jobs))

    for k in range(L, 0, -1):
        first = (1 << k) - 1
        span = 1 << (L - k)
        jobs = []
        for j in range(1 << k):
            node = first + j
            lo = int(leaf_offsets[j * span])
            hi = int(leaf_offsets[(j + 1) * span])
            if k == L:
                cand = np.arange(lo, hi, dtype=np.int64)
            else:
                cand = np.concatenate([skel[2 * node + 1], skel[2 * node + 2]])
            jobs.append((node, cand, lo, hi, X, h, n_samp, rank_rule, seed, full))
        for j, (sk, P) in enumerate(run_level(jobs)):
            skel[first + j] = sk
            pmat[first + j] = P
        if progress is not None:
            progress(f"skeletons of level {k} done ({1 << k} nodes)")

    skel[0] = np.zeros(0, dtype=np.int64)
    pmat[0] = np.zeros((0, 0))
    skel_offsets = np.zeros(n_nodes + 1, dtype=np.int64)
    p_offsets = np.zeros(n_nodes + 1, dtype=np.int64)
    for i in range(n_nodes):
        skel_offsets[i + 1] = skel_offsets[i] + skel[i].shape[0]
        p_offsets[i + 1] = p_offsets[i] + pmat[i].size
    skel_index = np.concatenate(skel).astype(np.int32)
    p_values = np.concatenate([p.ravel() for p in pmat]).astype(np.float64)
    return skel_offsets, skel_index, p_offsets, p_values
