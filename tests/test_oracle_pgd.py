"""Pins of the oracle's projected-gradient block solvers (oracle/pgd.py) against what the
mathematics fixes: the Lipschitz constant from the singular values of B, the descent
property of a 1/L projected gradient step, the r = 1 closed form, the NNLS solution from
an independent solver, its KKT conditions, and plain BCD with these solvers decreasing F."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle


def _block(seed, I=30, r=5, m=60):
    g = np.random.default_rng(seed)
    B = g.random((m, r))
    X = g.random((I, m))
    return X @ B, B.T @ B, B, g.random((I, r))


def _obj(W, P, G):
    return 0.5 * np.sum((W @ G) * W) - np.sum(P * W)


def test_lipschitz_is_the_largest_squared_singular_value():
    _, G, B, _ = _block(0)
    assert oracle.lipschitz(G) == pytest.approx(np.linalg.svd(B, compute_uv=False)[0] ** 2,
                                                rel=1e-12)


def test_projected_gradient_step_decreases_the_block_objective():
    P, G, _, W = _block(1)
    L = oracle.lipschitz(G)
    f = _obj(W, P, G)
    for _ in range(30):
        W = oracle.pg_step(W, P, G, L)
        assert W.min() >= 0.0
        f_new = _obj(W, P, G)
        assert f_new <= f + 1e-12 * abs(f)
        f = f_new


def test_rank_one_closed_form():
    g = np.random.default_rng(2)
    P = g.standard_normal((20, 1))
    G = np.array([[2.5]])
    W, s, _ = oracle.pgd(g.random((20, 1)), P, G, max_iters=1, tol=0.0)
    np.testing.assert_allclose(W, np.maximum(0.0, P / 2.5), rtol=1e-13, atol=1e-15)
    Wn, _, _ = oracle.nesterov(g.random((20, 1)), P, G, max_iters=1, tol=0.0)
    np.testing.assert_allclose(Wn, np.maximum(0.0, P / 2.5), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("solver,iters", [("pgd", 20000), ("nesterov", 3000)])
def test_converges_to_the_nnls_solution(solver, iters):
    P, G, _, W0 = _block(3, I=8, r=4)
    W, _, _ = getattr(oracle, solver)(W0, P, G, max_iters=iters, tol=0.0)
    # each row solves min_{w >= 0} 1/2 w^T G w - p^T w = 1/2 ||R w - R^{-T} p||^2 + const
    R = np.linalg.cholesky(G).T
    for i in range(P.shape[0]):
        ref, _ = nnls(R, np.linalg.solve(R.T, P[i]))
        np.testing.assert_allclose(W[i], ref, rtol=1e-6, atol=1e-8)
    grad = W @ G - P
    assert W.min() >= 0.0
    assert grad.min() >= -1e-6 * np.abs(P).max()
    assert np.abs(W * grad).max() <= 1e-6 * np.abs(P).max() * np.abs(W).max()


def test_first_nesterov_step_is_a_plain_step_and_dead_block_is_zero():
    P, G, _, W0 = _block(4)
    W1, _, _ = oracle.pgd(W0, P, G, max_iters=1, tol=0.0)
    N1, _, _ = oracle.nesterov(W0, P, G, max_iters=1, tol=0.0)
    np.testing.assert_array_equal(W1, N1)
    Wz, _, _ = oracle.pgd(W0, np.zeros_like(P), np.zeros_like(G), max_iters=3)
    assert not Wz.any()


def test_stopping_rule_counts():
    P, G, _, W0 = _block(5)
    _, s, d = oracle.pgd(W0, P, G, max_iters=7, tol=0.0)
    assert s == 7 and len(d) == 7
    _, s, d = oracle.pgd(W0, P, G, max_iters=500, tol=1e-2)
    assert s < 500 and d[-1] <= 1e-2 * d[0] and all(x > 1e-2 * d[0] for x in d[1:-1])


@pytest.mark.parametrize("inner", ["pgd", "nesterov"])
def test_plain_bcd_with_gradient_blocks_is_monotone(inner):
    """beta0 = 0: no extrapolation, so Algorithm 2 is plain BCD with a descent block solver
    and F decreases at every outer iteration; iterates stay nonnegative."""
    import synth
    pr = synth.make_problem((12, 10, 9), 3, snr_db=30.0, data_seed=3, init_seed=4)
    res = oracle.her_solve(pr.T, pr.A0, 15, params=oracle.HERParams(beta0=0.0, inner=inner))
    f = np.array([res.fhat0] + res.fhat)
    assert np.all(np.diff(f) <= 1e-12 * f[:-1])
    assert min(a.min() for a in res.factors) >= 0.0
    assert not any(res.restart)


# Momentum weights (t_{s-1} - 1) / t_s of the accelerated projected gradient with t_0 = 1,
# t_s = (1 + sqrt(1 + 4 t_{s-1}^2)) / 2 (Sec. 2.2, the reading of Nesterov-type
# acceleration): t_1 = (1 + sqrt 5) / 2 = 1.6180339887..., t_2 = 2.1935270853...,
# t_3 = 2.7497913401..., so the weights of the first four extrapolations are
# 0, 0.2817535251..., 0.4340427828..., 0.5310638054... (worked out by hand once and stored
# as numbers, not recomputed from the recurrence).
_NESTEROV_WEIGHTS = (0.0, 0.28175352512532087, 0.434042782780302, 0.5310638054044795)


def _diag_accelerated_closed_form(w0, p, g, L, weights):
    """Accelerated projected gradient on a diagonal G with the projection inactive: every
    entry follows x_{s+1} = (1 - g/L) y_s + p/L, y_s = x_s + c_s (x_s - x_{s-1}), y_0 = x_0."""
    a = 1.0 - g / L
    x_prev, x = None, w0.copy()
    y = x.copy()
    out = []
    for c in weights:
        x_new = a * y + p / L
        out.append(x_new)
        x_prev, x = x, x_new
        y = x + c * (x - x_prev)
    return out


def test_nesterov_momentum_weights_closed_form():
    """Four accelerated steps on a diagonal G (projection inactive) equal the closed form with
    the stored weights; the two plausible slips of the recurrence, the weight
    (t_s - 1) / t_s and t advanced before the extrapolation, both miss it."""
    g = np.array([4.0, 1.0, 2.5, 0.6])
    G = np.diag(g)
    P = np.array([[8.0, 3.0, 5.0, 1.5], [4.0, 2.0, 9.0, 0.7]])
    W0 = np.array([[1.0, 0.5, 0.2, 0.3], [0.1, 2.0, 1.0, 0.05]])
    L = 4.0
    assert oracle.lipschitz(G) == L
    ref = _diag_accelerated_closed_form(W0, P, g, L, _NESTEROV_WEIGHTS)
    assert min(x.min() for x in ref) > 0.0  # projection inactive throughout
    for steps in (1, 2, 3, 4):
        W, s, _ = oracle.nesterov(W0, P, G, max_iters=steps, tol=0.0)
        assert s == steps
        np.testing.assert_allclose(W, ref[steps - 1], rtol=1e-14, atol=1e-14)
    # the mutated recurrences give visibly different iterates at step 3 or 4
    t = [1.0, 1.618033988749895, 2.193527085331054, 2.749791340120445, 3.2948796779470473]
    slip_weight = [(t[s + 1] - 1.0) / t[s + 1] for s in range(4)]
    slip_order = [(t[s + 1] - 1.0) / t[s + 2] for s in range(3)] + [0.0]
    for wrong in (slip_weight, slip_order):
        bad = _diag_accelerated_closed_form(W0, P, g, L, wrong)
        assert np.abs(bad[3] - ref[3]).max() > 1e-3
