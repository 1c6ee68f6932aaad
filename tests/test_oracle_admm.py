"""Pins of the oracle's ADMM block solver (Sec. 2.1.2, reading in oracle/admm.py) against
closed forms and an independent NNLS solver."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import synth


def test_diagonal_gram_closed_form():
    """Diagonal G = diag(g) decouples the columns; with positive targets P/g and a positive
    start the projection and the dual stay inactive, so every column contracts to P/g by
    the factor rho / (g + rho) per step with rho = mean(g):
    Z_s = P/g + (Z_0 - P/g) (rho / (g + rho))^s."""
    g = np.array([1.0, 2.0, 4.0, 8.0])
    rho = g.mean()
    P = np.array([[3.0, 1.0, 8.0, 4.0], [0.5, 6.0, 2.0, 16.0]])
    Z0 = np.array([[1.0, 2.0, 0.5, 3.0], [2.0, 1.0, 1.0, 1.0]])
    for s in (1, 2, 5):
        Z, steps, _ = oracle.admm(Z0, P, np.diag(g), max_iters=s, tol=-1.0)
        assert steps == s
        want = P / g + (Z0 - P / g) * (rho / (g + rho)) ** s
        assert np.allclose(Z, want, rtol=1e-14, atol=1e-14)


def test_negative_target_scalar_sequence():
    """r = 1, G = 2 (rho = 2), P = -6, Z_0 = 1, worked by hand from the three updates:
    W_1 = -1, Z_1 = 0, U_1 = -1; W_2 = -1, Z_2 = 0, U_2 = -2; then U_s = -3 + 2^(2-s) -> -3,
    the negated KKT multiplier (6) over rho. A sign slip in the dual update or in the
    W-update's right-hand side changes these numbers."""
    for s, u in [(1, -1.0), (2, -2.0), (3, -2.5), (4, -2.75), (6, -3.0 + 2.0 ** -4)]:
        Z, steps, _, U = oracle.admm(np.array([[1.0]]), np.array([[-6.0]]), np.array([[2.0]]),
                                     max_iters=s, tol=-1.0, return_dual=True)
        assert steps == s
        assert Z[0, 0] == 0.0
        assert U[0, 0] == pytest.approx(u, abs=1e-15)


def test_converges_to_the_nnls_solution():
    """Many steps reach the NNLS solution of each row (scipy's active-set NNLS on the
    Cholesky form of the normal equations), which satisfies the KKT conditions."""
    rng = np.random.default_rng(3)
    B = rng.random((60, 5))
    M = rng.random((7, 60)) - 0.3
    P, G = M @ B, B.T @ B
    W0 = rng.random((7, 5))
    Z, _, _ = oracle.admm(W0, P, G, max_iters=4000, tol=-1.0)
    C = np.linalg.cholesky(G).T
    for i in range(7):
        ref, _ = nnls(C, np.linalg.solve(C.T, P[i]))
        assert np.allclose(Z[i], ref, atol=1e-8)
    grad = Z @ G - P
    assert Z.min() >= 0 and grad.min() >= -1e-7 and np.abs(Z * grad).max() <= 1e-7


def test_stopping_rule_and_dead_block():
    rng = np.random.default_rng(4)
    B = rng.random((40, 4))
    P, G = rng.random((6, 40)) @ B, B.T @ B
    Z, s, d = oracle.admm(rng.random((6, 4)), P, G, max_iters=50, tol=1e-2)
    assert len(d) == s
    assert s == 50 or d[-1] <= 1e-2 * d[0]
    assert all(x > 1e-2 * d[0] for x in d[1:-1])
    Z, s, _ = oracle.admm(np.ones((3, 2)), np.zeros((3, 2)), np.zeros((2, 2)))
    assert np.array_equal(Z, np.zeros((3, 2)))


@pytest.mark.slow
def test_her_admm_improves_on_ao_admm():
    """HER with ADMM blocks (HER-ADMM) reaches a lower objective than the same blocks
    without extrapolation (beta0 = 0) on the 50^3 r = 10 workload (the paper's comparison
    of HER-ADMM with AO-ADMM, direction only); every iterate stays nonnegative."""
    pr = synth.workload("cube50_r10")
    T = pr.T.astype(np.float32).astype(np.float64)
    A0 = [a.astype(np.float32).astype(np.float64) for a in pr.A0]
    her = oracle.her_solve(T, A0, 60, oracle.HERParams(inner="admm"))
    ao = oracle.her_solve(T, A0, 60, oracle.HERParams(inner="admm", beta0=0.0))
    assert oracle.objective(T, her.factors) < oracle.objective(T, ao.factors)
    assert min(a.min() for a in her.factors) >= 0
