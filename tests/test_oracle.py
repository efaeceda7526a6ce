"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code path:
  * the kernel against its closed form (eq. (1)) written out with math.exp;
  * the whole solve against dense LAPACK on the assembled lambda*I + K~;
  * the exact case s = |node| (every P a permutation, K~ = K) against a dense
    solve with K built entry by entry;
  * one leaf (L = 0) = dense LU; one split (L = 1) = an explicit
    Sherman-Morrison-Woodbury step (eq. (5)) with D, U, V of eq. (8);
  * the residual bound ||(lambda I + K~) x - b|| / ||b|| <= 1e-12 and the
    eps_I invariant of eq. (17);
  * a zero pivot (duplicated point, lambda = 0) is reported.
"""
import math
import types

import numpy as np
import pytest

import oracle
from paper_1602_01376_amd.setup import make_problem


def _kernel_by_hand(X, h):
    n = X.shape[0]
    K = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            d2 = 0.0
            for t in range(X.shape[1]):
                diff = float(X[i, t]) - float(X[j, t])
                d2 += diff * diff
            K[i, j] = math.exp(-0.5 * d2 / (h * h))
    return K


def test_kernel_closed_form():
    # K(x, x) = 1 and K at ||x - y|| = 5, h = 5 is exp(-1/2).
    x = np.array([[0.0, 0.0]])
    y = np.array([[3.0, 4.0]])
    assert oracle.gaussian(x, x, 0.7)[0, 0] == 1.0
    assert abs(oracle.gaussian(x, y, 5.0)[0, 0] - math.exp(-0.5)) < 1e-16
    # squared distance 2 h^2 gives exp(-1); the 1/2 of eq. (1) matters
    z = np.array([[1.0, 1.0]])
    assert abs(oracle.gaussian(x, z, 1.0)[0, 0] - math.exp(-1.0)) < 1e-16
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, 3))
    np.testing.assert_allclose(oracle.gaussian(X, X, 1.3), _kernel_by_hand(X, 1.3),
                               rtol=1e-14, atol=1e-15)


def test_setup_invariants():
    pb = make_problem("susy", n=1 << 13, depth=5)
    sizes = np.diff(pb.leaf_offsets)
    assert sizes.min() >= 64 and sizes.max() <= 512 and sizes.sum() == pb.n
    assert np.array_equal(np.sort(pb.perm), np.arange(pb.n))
    for node in range(1, pb.n_nodes):
        sk = pb.skel(node)
        a, b = pb.node_range(node)
        assert np.all((sk >= a) & (sk < b))
        if not pb.is_leaf(node):
            cand = np.concatenate([pb.skel(2 * node + 1), pb.skel(2 * node + 2)])
            assert set(sk.tolist()) <= set(cand.tolist())
            cols = [int(np.where(cand == v)[0][0]) for v in sk]
        else:
            cols = [int(v - a) for v in sk]
        P = pb.P(node)
        np.testing.assert_array_equal(P[:, cols], np.eye(len(sk)))
        assert 32 <= len(sk) <= 256
    pb2 = make_problem("susy", n=1 << 13, depth=5)
    assert np.array_equal(pb.skel_index, pb2.skel_index)
    assert np.array_equal(pb.p_values, pb2.p_values)


def test_single_leaf_is_dense_lu():
    pb = make_problem("tiny", n=200, depth=0)
    lam = 1e-2
    b = np.random.default_rng(1).standard_normal(200)
    F = oracle.factorize(pb, lam)
    A = _kernel_by_hand(pb.X, pb.h) + lam * np.eye(200)
    np.testing.assert_allclose(oracle.solve(F, b), np.linalg.solve(A, b), rtol=1e-10)


def _hand_problem():
    """Two leaves of three 2-d points, one skeleton each, P chosen by hand."""
    X = np.array([[0.0, 0.0], [0.4, 0.1], [0.2, 0.5],
                  [1.5, 1.0], [1.1, 1.3], [1.8, 0.7]])
    return types.SimpleNamespace(
        X=X, depth=1, h=0.8,
        leaf_offsets=np.array([0, 3, 6]),
        skel_offsets=np.array([0, 0, 1, 2]),
        skel_index=np.array([1, 4], dtype=np.int32),
        p_offsets=np.array([0, 0, 3, 6]),
        p_values=np.array([0.7, 1.0, -0.2, 0.3, 1.0, 0.9]))


def test_one_split_is_one_woodbury_step():
    pb = _hand_problem()
    lam = 0.05
    b = np.array([1.0, -2.0, 0.5, 0.25, 3.0, -1.0])
    X, h = pb.X, pb.h
    K = _kernel_by_hand(X, h)
    Pl = np.array([[0.7, 1.0, -0.2]])      # P_{l~ l}, skeleton = point 1
    Pr = np.array([[0.3, 1.0, 0.9]])       # P_{r~ r}, skeleton = point 4
    D = K.copy()
    D[:3, 3:] = 0.0
    D[3:, :3] = 0.0
    D += lam * np.eye(6)
    U = np.zeros((6, 2))
    U[:3, 0] = K[:3, 4]                    # K_{l r~}
    U[3:, 1] = K[3:, 1]                    # K_{r l~}
    V = np.zeros((2, 6))
    V[0, 3:] = Pr[0]
    V[1, :3] = Pl[0]
    Dinv = np.linalg.inv(D)
    W = Dinv @ U
    Z = np.linalg.inv(np.eye(2) + V @ W)
    x_smw = (np.eye(6) - W @ Z @ V) @ Dinv @ b          # eq. (5)
    x_dense = np.linalg.solve(D + U @ V, b)
    np.testing.assert_allclose(x_smw, x_dense, rtol=1e-12)
    F = oracle.factorize(pb, lam)
    np.testing.assert_allclose(oracle.solve(F, b), x_smw, rtol=1e-12)
    Kt = oracle.dense_assemble(pb)
    np.testing.assert_allclose(Kt + lam * np.eye(6), D + U @ V, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(oracle.matvec(pb, lam, b), (D + U @ V) @ b, rtol=1e-13)


def test_full_skeletons_give_exact_kernel():
    pb = make_problem("tiny", n=256, depth=3, full_skeletons=True)
    lam = 1e-2
    K = _kernel_by_hand(pb.X, pb.h)
    np.testing.assert_allclose(oracle.dense_assemble(pb), K, rtol=1e-14, atol=1e-15)
    b = np.random.default_rng(2).standard_normal((256, 3))
    A = K + lam * np.eye(256)
    F = oracle.factorize(pb, lam)
    x = oracle.solve(F, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(oracle.matvec(pb, lam, b), A @ b, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("workload,n,depth", [("tiny", 1024, 3), ("susy", 2048, 3),
                                               ("covtype", 1024, 2)])
def test_solve_matches_dense_lu(workload, n, depth):
    pb = make_problem(workload, n=n, depth=depth)
    lam = pb.lam
    Kt = oracle.dense_assemble(pb)
    A = Kt + lam * np.eye(n)
    b = np.random.default_rng(3).standard_normal((n, 2))
    x_dense = np.linalg.solve(A, b)
    F = oracle.factorize(pb, lam)
    x = oracle.solve(F, b)
    kappa = np.linalg.cond(A)
    rel = np.linalg.norm(x - x_dense) / np.linalg.norm(x_dense)
    assert rel <= max(1e-13, 50 * kappa * np.finfo(float).eps), (rel, kappa)
    # two independent constructions of K~: block assembly vs the Evaluate traversal
    np.testing.assert_allclose(oracle.matvec(pb, lam, b), A @ b, rtol=1e-11,
                               atol=1e-11 * np.abs(A @ b).max())


def test_residual_and_eps_I_on_tiny_workload():
    pb = make_problem("tiny")
    lam = pb.lam
    b = np.random.default_rng(4).standard_normal(pb.n)
    F = oracle.factorize(pb, lam)
    x = oracle.solve(F, b)
    res = np.linalg.norm(oracle.matvec(pb, lam, x) - b) / np.linalg.norm(b)
    assert res <= 1e-12, res
    w = np.random.default_rng(5).standard_normal(pb.n)
    eps_I = np.linalg.norm(w - oracle.solve(F, oracle.matvec(pb, lam, w))) / np.linalg.norm(w)
    assert eps_I <= 1e-11, eps_I


def test_matvec_rows_match_matvec():
    pb = make_problem("susy", n=4096, depth=4)
    x = np.random.default_rng(6).standard_normal((pb.n, 2))
    y = oracle.matvec(pb, 1e-3, x)
    rows = [0, 1, 77, 2048, 4095]
    np.testing.assert_allclose(oracle.matvec_rows(pb, 1e-3, x, rows), y[rows], rtol=1e-12)


def test_skeletonize_weights_select_points_with_full_skeletons():
    # With s = |node| at every node each P is a permutation onto the node's
    # skeleton order, so the Skeletonize weights are the values of x at the
    # skeleton points themselves: q_c = x[skel(c)] (leaf and internal nodes).
    pb = make_problem("tiny", n=256, depth=3, full_skeletons=True)
    x = np.random.default_rng(8).standard_normal((256, 2))
    q = oracle.skeletonize_weights(pb, x)
    for node in range(1, pb.n_nodes):
        np.testing.assert_allclose(q[node], x[pb.skel(node)], rtol=0, atol=1e-15)
    # the hand problem: one skeleton point per leaf, P written out
    hp = _hand_problem()
    xh = np.arange(1.0, 7.0)
    qh = oracle.skeletonize_weights(hp, xh)
    assert abs(qh[1][0] - (0.7 * 1 + 1.0 * 2 - 0.2 * 3)) < 1e-14
    assert abs(qh[2][0] - (0.3 * 4 + 1.0 * 5 + 0.9 * 6)) < 1e-14


def test_skeleton_projection_of_corrected_solution():
    # After w = v - W Z V v at node a, the children's skeleton projections of
    # w equal y = Z (V v):  V w = V v - V W y = V v - (Z^-1 - I) y = y.
    pb = make_problem("tiny", n=1024, depth=3)
    F = oracle.factorize(pb, pb.lam)
    u = np.random.default_rng(7).standard_normal(pb.n)
    node, l, r = 0, 1, 2
    nl = pb.node_range(l)[1]
    v_l = oracle.solve_node(F, l, u[:nl])
    v_r = oracle.solve_node(F, r, u[nl:])
    w = oracle.solve_node(F, node, u)
    t = np.concatenate([F.Pfull[r] @ v_r, F.Pfull[l] @ v_l])
    import scipy.linalg as sla
    y = sla.lu_solve(F.Z[node], t)
    s_r = F.Pfull[r].shape[0]
    np.testing.assert_allclose(F.Pfull[r] @ w[nl:], y[:s_r], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(F.Pfull[l] @ w[:nl], y[s_r:], rtol=1e-9, atol=1e-11)


def test_zero_pivot_is_reported():
    pb = make_problem("tiny", n=256, depth=2)
    pb.X[1] = pb.X[0]            # two equal rows in the first leaf's block
    with pytest.raises(oracle.OracleSingular) as ei:
        oracle.factorize(pb, 0.0)
    assert ei.value.node == 3 and ei.value.what == "leaf block"
