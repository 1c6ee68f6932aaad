"""Pins for the oracle's A-HALS block solver.

Checks: the optimality (KKT) conditions of each one-column NNLS, monotone decrease of the
block objective, the rank-one closed form, convergence to the NNLS solution computed by
scipy.optimize.nnls (a library routine), the stopping rule, and the dead-component case.
"""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle


def _block_problem(seed=0, dims=(6, 7, 8), r=4, n=0):
    g = np.random.default_rng(seed)
    A = [g.random((I, r)) for I in dims]
    T = oracle.kruskal([g.random((I, r)) for I in dims]) + 0.05 * g.random(dims)
    P = oracle.mttkrp(T, A, n)
    G = oracle.hadamard_gram(A, n)
    return T, A, P, G


def _block_objective(T, A, n, W):
    B = [a for a in A]
    B = B[:n] + [W] + B[n + 1:]
    return oracle.objective(T, B)


def test_column_update_satisfies_kkt():
    T, A, P, G = _block_problem()
    W = A[0].copy()
    scale = np.abs(P).max()
    for j in range(W.shape[1]):
        oracle.hals_column(W, P, G, j)
        g = W @ G[:, j] - P[:, j]       # gradient of the block objective w.r.t. W[:, j]
        assert np.all(W[:, j] >= 0)
        assert np.all(g >= -1e-12 * scale)
        assert np.allclose(W[:, j] * g, 0.0, atol=1e-12 * scale * max(1.0, W.max()))


def test_every_column_update_does_not_increase_objective():
    T, A, P, G = _block_problem(seed=1, n=1)
    W = A[1].copy()
    f = _block_objective(T, A, 1, W)
    for _ in range(3):
        for j in range(W.shape[1]):
            oracle.hals_column(W, P, G, j)
            f_new = _block_objective(T, A, 1, W)
            assert f_new <= f * (1 + 1e-12)
            f = f_new


def test_rank_one_is_projected_ratio():
    g = np.random.default_rng(2)
    P = g.standard_normal((9, 1))
    G = np.array([[2.5]])
    W, s, _ = oracle.hals(g.random((9, 1)), P, G, max_sweeps=5, tol=0.0)
    assert np.allclose(W, np.maximum(0.0, P / 2.5), rtol=1e-15)
    assert s == 2  # the second sweep changes nothing and stops the tol = 0 run


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_many_sweeps_reach_the_nnls_solution(seed):
    """Each row solves min_{w>=0} 1/2 w^T G w - p^T w = 1/2 ||L^T w - L^{-1} p||^2 + const
    with G = L L^T; scipy's nnls solves that least-squares form."""
    T, A, P, G = _block_problem(seed=seed, r=5, n=2)
    W, _, _ = oracle.hals(A[2], P, G, max_sweeps=3000, tol=0.0)
    L = np.linalg.cholesky(G)
    for i in range(W.shape[0]):
        x, _ = nnls(L.T, np.linalg.solve(L, P[i]))
        assert np.allclose(W[i], x, rtol=1e-7, atol=1e-9)


def test_stopping_rule_sweeps_and_deltas():
    T, A, P, G = _block_problem(seed=3, dims=(20, 9, 10), r=6)
    W0 = A[0]
    W, s, d = oracle.hals(W0, P, G, max_sweeps=50, tol=1e-2)
    assert len(d) == s
    if s < 50:
        assert d[-1] <= 1e-2 * d[0]
    assert all(x > 1e-2 * d[0] for x in d[1:-1])
    # same result as running exactly s sweeps without the rule
    W_fixed, s_fixed, _ = oracle.hals(W0, P, G, max_sweeps=s, tol=0.0)
    assert s_fixed == s and np.array_equal(W, W_fixed)
    # the recorded deltas are the Frobenius norms of consecutive sweep differences
    prev = np.array(W0, dtype=float)
    for k in range(1, min(s, 4) + 1):
        cur, _, _ = oracle.hals(W0, P, G, max_sweeps=k, tol=0.0)
        assert np.isclose(np.linalg.norm(cur - prev), d[k - 1], rtol=1e-12)
        prev = cur


def test_dead_component_stays_zero():
    g = np.random.default_rng(4)
    dims, r = (5, 6, 7), 3
    A = [g.random((I, r)) for I in dims]
    A[1][:, 2] = 0.0           # component 2 is dead in another factor
    T = g.random(dims)
    P = oracle.mttkrp(T, A, 0)
    G = oracle.hadamard_gram(A, 0)
    assert G[2, 2] == 0.0 and np.all(P[:, 2] == 0.0)
    W, _, _ = oracle.hals(A[0], P, G, max_sweeps=10, tol=0.0)
    assert np.all(W[:, 2] == 0.0) and np.all(np.isfinite(W))
