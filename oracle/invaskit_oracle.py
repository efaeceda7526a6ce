"""Plain FP64 CPU oracle for the INV-ASKIT factorization and solve.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the HIP
path and imports nothing from the product package: a problem is passed in as
any object carrying the arrays X, depth, leaf_offsets, skel_offsets,
skel_index, p_offsets, p_values and the bandwidth h (tree order, heap node
numbering: root 0, children of i are 2i+1 and 2i+2).

What it computes, following the paper (Yu, March, Xiao, Biros, "INV-ASKIT:
A Parallel Fast Direct Solver for Kernel Matrices"):

  gaussian          the kernel of eq. (1), by direct differences
  factorize         Algorithm 1 (post-order Factorize), with the block forms
                    of eqs. (10) and (11) and the full P of
                    eq. (12)
  solve             Algorithm 2 (Solve), w = v - W Z V v per internal node
  matvec            the Skeletonize upward pass and the Evaluate traversal of
                    Section II-B with separation "i not in alpha", which is
                    exactly lambda*I + K~ (eqs. (3),
                    (7))
  dense_assemble    K~ written out block by block from eqs.
                    (3), (7), (8)

Readings where the paper is silent: lambda sits only on the diagonal of the
leaf blocks (the paper calls the extension to lambda*I + K trivial); the
reduced system keeps the paper's block order, r~ rows first; the root has no
skeleton; P of an internal node has columns [l~ | r~].

Pins: every function here is checked by tests marked "not gpu" against
closed forms, dense LAPACK on the assembled matrix, the exact case s = |node|
(K~ = K), the one-leaf and one-split special cases, and residual bounds.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.spatial.distance import cdist


class OracleSingular(RuntimeError):
    """Raised when a leaf block or a reduced system has a zero pivot."""

    def __init__(self, node, what):
        super().__init__(f"singular {what} at node {node}")
        self.node = node
        self.what = what


# ---------------------------------------------------------------- tree access
def _level(node):
    return int(math.floor(math.log2(node + 1)))


def _range(pb, node):
    k = _level(node)
    j = node - ((1 << k) - 1)
    span = 1 << (pb.depth - k)
    return int(pb.leaf_offsets[j * span]), int(pb.leaf_offsets[(j + 1) * span])


def _is_leaf(pb, node):
    return _level(node) == pb.depth


def _skel(pb, node):
    return np.asarray(pb.skel_index[pb.skel_offsets[node]:pb.skel_offsets[node + 1]],
                      dtype=np.int64)


def _P(pb, node):
    s = int(pb.skel_offsets[node + 1] - pb.skel_offsets[node])
    a, b = int(pb.p_offsets[node]), int(pb.p_offsets[node + 1])
    return np.asarray(pb.p_values[a:b], dtype=np.float64).reshape(s, -1)


# --------------------------------------------------------------------- kernel
def gaussian(XA, XB, h):
    """K(x, y) = exp(-||x - y||^2 / (2 h^2)), eq. (1), in FP64 with
    squared distances taken by direct differences."""
    A = np.asarray(XA, dtype=np.float64)
    B = np.asarray(XB, dtype=np.float64)
    return np.exp(-0.5 * cdist(A, B, "sqeuclidean") / (h * h))


def _lu(A, node, what):
    lu, piv = sla.lu_factor(A, check_finite=False, overwrite_a=True)
    dg = np.diag(lu)
    if not np.all(np.isfinite(dg)) or np.any(dg == 0.0):
        raise OracleSingular(node, what)
    return lu, piv


# ------------------------------------------------------------- factorization
class Factorization:
    """Holds, per node: leaf LU (leaves), W (non-root nodes: W_c =
    Kt_cc^-1 K_{c, sibling skeleton}), the LU of the reduced system
    (internal nodes) and the full P_{c~ c} (non-root nodes)."""

    def __init__(self, pb, lam):
        self.pb = pb
        self.lam = float(lam)
        self.leaf_lu = {}
        self.W = {}
        self.Z = {}
        self.Pfull = {}


def factorize(pb, lam):
    """Algorithm 1, Factorize(root), as a post-order recursion.

    Leaf: LU with partial pivoting of lambda*I + K_aa.  Internal node a with
    children l, r: factor both children; form K_{l r~}, K_{r l~} and the full
    P_{l~ l}, P_{r~ r} (eq. (12)); W_{l r~} = Solve(l, K_{l r~}) and
    W_{r l~} = Solve(r, K_{r l~}); LU of the reduced system
    [[I, P_{r~r} W_{r l~}], [P_{l~l} W_{l r~}, I]] of eq. (11).
    """
    F = Factorization(pb, lam)
    X = pb.X

    def full_p(node):
        # eq. (12): P_{a~ a} = P_{a~[l~ r~]} blkdiag(P_{l~ l}, P_{r~ r});
        # leaves store P_{a~ a} directly.
        if _is_leaf(pb, node):
            return _P(pb, node)
        l, r = 2 * node + 1, 2 * node + 2
        Pa = _P(pb, node)
        sl = F.Pfull[l].shape[0]
        return np.hstack([Pa[:, :sl] @ F.Pfull[l], Pa[:, sl:] @ F.Pfull[r]])

    def fac(node):
        if _is_leaf(pb, node):
            a, b = _range(pb, node)
            A = gaussian(X[a:b], X[a:b], pb.h)
            A[np.diag_indices_from(A)] += F.lam
            F.leaf_lu[node] = _lu(A, node, "leaf block")
        else:
            l, r = 2 * node + 1, 2 * node + 2
            fac(l)
            fac(r)
            la, lb = _range(pb, l)
            ra, rb = _range(pb, r)
            K_lr = gaussian(X[la:lb], X[_skel(pb, r)], pb.h)   # K_{l r~}
            K_rl = gaussian(X[ra:rb], X[_skel(pb, l)], pb.h)   # K_{r l~}
            F.W[l] = solve_node(F, l, K_lr)                     # W_{l r~}
            F.W[r] = solve_node(F, r, K_rl)                     # W_{r l~}
            s_l, s_r = F.Pfull[l].shape[0], F.Pfull[r].shape[0]
            Zm = np.zeros((s_r + s_l, s_r + s_l))
            Zm[:s_r, :s_r] = np.eye(s_r)
            Zm[s_r:, s_r:] = np.eye(s_l)
            Zm[:s_r, s_r:] = F.Pfull[r] @ F.W[r]                # P_{r~r} W_{r l~}
            Zm[s_r:, :s_r] = F.Pfull[l] @ F.W[l]                # P_{l~l} W_{l r~}
            F.Z[node] = _lu(Zm, node, "reduced system")
        if node != 0:
            F.Pfull[node] = full_p(node)

    fac(0)
    return F


def solve_node(F, node, U):
    """Algorithm 2, w = Solve(node, U): applies (lambda*I + K~_{node,node})^-1
    to the rows of U owned by `node` (U has one row per point of the node).

    Leaf: LU solve.  Internal: v_l = Solve(l, U_l), v_r = Solve(r, U_r);
    w = v - W Z V v with the blocks of eq. (11):
    t = [P_{r~r} v_r ; P_{l~l} v_l], y = Z^-1 t,
    w_l = v_l - W_{l r~} y[:s_r], w_r = v_r - W_{r l~} y[s_r:].
    """
    pb = F.pb
    U = np.asarray(U, dtype=np.float64)
    if _is_leaf(pb, node):
        return sla.lu_solve(F.leaf_lu[node], U, check_finite=False)
    l, r = 2 * node + 1, 2 * node + 2
    la, lb = _range(pb, l)
    nl = lb - la
    v_l = solve_node(F, l, U[:nl])
    v_r = solve_node(F, r, U[nl:])
    s_r = F.Pfull[r].shape[0]
    t = np.concatenate([F.Pfull[r] @ v_r, F.Pfull[l] @ v_l], axis=0)
    y = sla.lu_solve(F.Z[node], t, check_finite=False)
    w_l = v_l - F.W[l] @ y[:s_r]
    w_r = v_r - F.W[r] @ y[s_r:]
    return np.concatenate([w_l, w_r], axis=0)


def solve(F, b):
    """x = (lambda*I + K~)^-1 b for b of shape (N,) or (N, r)."""
    return solve_node(F, 0, b)


# ------------------------------------------------------------------- matvec
def skeletonize_weights(pb, x):
    """Skeletonize, weight part: q_a = P_{a~ a} x_a for a leaf and
    q_a = P_{a~[l~ r~]} [q_l ; q_r] for an internal node (upward pass)."""
    x = np.asarray(x, dtype=np.float64)
    q = {}
    for k in range(pb.depth, 0, -1):
        for node in range((1 << k) - 1, (1 << (k + 1)) - 1):
            if k == pb.depth:
                a, b = _range(pb, node)
                q[node] = _P(pb, node) @ x[a:b]
            else:
                q[node] = _P(pb, node) @ np.concatenate(
                    [q[2 * node + 1], q[2 * node + 2]], axis=0)
    return q


def matvec(pb, lam, x):
    """y = (lambda*I + K~) x by the Evaluate traversal: a target i separated
    from node a (i not in a) takes K_{i a~} q_a; a leaf containing i adds
    K_{i a} x_a exactly; lambda*x is the regularization."""
    x = np.asarray(x, dtype=np.float64)
    q = skeletonize_weights(pb, x)
    y = lam * x.copy()
    X = pb.X

    def evaluate(node, ta, tb):
        # targets [ta, tb) all lie inside `node` here
        if _is_leaf(pb, node):
            y[ta:tb] += gaussian(X[ta:tb], X[ta:tb], pb.h) @ x[ta:tb]
            return
        l, r = 2 * node + 1, 2 * node + 2
        la, lb = _range(pb, l)
        ra, rb = _range(pb, r)
        # targets of r are separated from l, and vice versa
        y[ra:rb] += gaussian(X[ra:rb], X[_skel(pb, l)], pb.h) @ q[l]
        y[la:lb] += gaussian(X[la:lb], X[_skel(pb, r)], pb.h) @ q[r]
        evaluate(l, la, lb)
        evaluate(r, ra, rb)

    evaluate(0, 0, pb.X.shape[0])
    return y


def matvec_rows(pb, lam, x, rows, q=None):
    """Rows `rows` of (lambda*I + K~) x, each computed on its own from the
    Evaluate traversal (for spot checks at sizes where the full product is
    too slow).  `q` may carry precomputed skeleton weights."""
    x = np.asarray(x, dtype=np.float64)
    if q is None:
        q = skeletonize_weights(pb, x)
    X = pb.X
    out = []
    for i in rows:
        i = int(i)
        acc = lam * np.atleast_1d(x[i]).astype(np.float64)
        node = 0
        while not _is_leaf(pb, node):
            l, r = 2 * node + 1, 2 * node + 2
            la, lb = _range(pb, l)
            inside, other = (l, r) if la <= i < lb else (r, l)
            acc = acc + (gaussian(X[i:i + 1], X[_skel(pb, other)], pb.h) @ q[other]).reshape(-1)
            node = inside
        a, b = _range(pb, node)
        acc = acc + (gaussian(X[i:i + 1], X[a:b], pb.h) @ x[a:b]).reshape(-1)
        out.append(acc)
    return np.array(out).reshape((len(rows),) + x.shape[1:])


# ------------------------------------------------------------ dense assembly
def dense_assemble(pb):
    """K~ as a dense N x N matrix (tiny N only): leaf diagonal blocks are
    exact, and for every internal node with children l, r the blocks are
    K~[l, r] = K_{l r~} P_{r~ r} and K~[r, l] = K_{r l~} P_{l~ l}
    (eqs. (7), (8)), with the full P built level by
    level as stated in eq. (12)."""
    N = pb.X.shape[0]
    X = pb.X
    Kt = np.zeros((N, N))
    pf = {}
    for k in range(pb.depth, 0, -1):
        for node in range((1 << k) - 1, (1 << (k + 1)) - 1):
            if k == pb.depth:
                pf[node] = _P(pb, node)
            else:
                l, r = 2 * node + 1, 2 * node + 2
                pf[node] = _P(pb, node) @ sla.block_diag(pf[l], pf[r])
    for node in range((1 << pb.depth) - 1, (1 << (pb.depth + 1)) - 1):
        a, b = _range(pb, node)
        Kt[a:b, a:b] = gaussian(X[a:b], X[a:b], pb.h)
    for node in range(0, (1 << pb.depth) - 1):
        l, r = 2 * node + 1, 2 * node + 2
        la, lb = _range(pb, l)
        ra, rb = _range(pb, r)
        Kt[la:lb, ra:rb] = gaussian(X[la:lb], X[_skel(pb, r)], pb.h) @ pf[r]
        Kt[ra:rb, la:lb] = gaussian(X[ra:rb], X[_skel(pb, l)], pb.h) @ pf[l]
    return Kt
