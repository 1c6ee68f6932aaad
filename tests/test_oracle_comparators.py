"""Pins of the oracle's comparison algorithms (APG, iBPG, Bro's block-wise extrapolation;
oracle/comparators.py) against special cases that reduce to pinned parts, hand-worked
numbers and invariants."""
import numpy as np
import pytest

import oracle
import synth


def _problem(seed=0, dims=(12, 10, 9), r=3):
    pr = synth.make_problem(dims, r, snr_db=30.0, data_seed=seed, init_seed=seed + 1)
    return pr.T.astype(np.float64), [a.astype(np.float64) for a in pr.A0]


def _pg_sweep(T, A):
    """One block projected-gradient sweep (Algorithm 1 with one step per block), composed
    from the pinned Gram, MTTKRP, Lipschitz and step functions."""
    A = [a.copy() for a in A]
    for i in range(T.ndim):
        G = oracle.hadamard_gram(A, i)
        P = oracle.mttkrp(T, A, i)
        A[i] = oracle.pg_step(A[i], P, G, oracle.lipschitz(G))
    return A


def test_t_sequence_weights():
    """w_hat_{k-1} = (t_{k-1} - 1) / t_k from t_0 = 1: 0, 0.28175, 0.43404, 0.53106 (the
    numbers of the accelerated gradient's momentum weights)."""
    t, got = 1.0, []
    for _ in range(4):
        tn = oracle.t_next(t)
        got.append((t - 1.0) / tn)
        t = tn
    # t_1 = (1 + sqrt 5) / 2 = 1.618034, t_2 = 2.193527, t_3 = 2.749791, t_4 = 3.294880
    assert np.allclose(got, [0.0, 0.28175, 0.43404, 0.53106], atol=1e-5)


def test_apg_without_extrapolation_is_the_block_gradient_sweep():
    T, A0 = _problem(1)
    res = oracle.apg_solve(T, A0, 6, delta_w=0.0, keep_history=True)
    A = [a.copy() for a in A0]
    for k in range(6):
        A = _pg_sweep(T, A)
        for a, b in zip(A, res.history[k]):
            assert np.array_equal(a, b)
    assert not any(res.restart)


def test_apg_is_monotone_and_its_restart_redoes_the_sweep():
    """The restart makes every accepted iterate no worse than the previous one; a restarted
    iteration equals the plain gradient sweep from the previous iterate."""
    T, A0 = _problem(2, dims=(20, 18, 16), r=4)
    res = oracle.apg_solve(T, A0, 60, keep_history=True)
    f = [res.f0] + res.objective
    assert all(b <= a * (1 + 1e-12) for a, b in zip(f, f[1:]))
    assert all(w == 0.0 for w in res.weights[0])
    ks = [k for k, r in enumerate(res.restart) if r and k > 0]
    assert ks, "the seed should exercise the restart"
    k = ks[0]
    redo = _pg_sweep(T, res.history[k - 1])
    for a, b in zip(redo, res.history[k]):
        assert np.allclose(a, b, rtol=0, atol=0)
    for a in res.factors:
        assert a.min() >= 0


def test_ibpg_block_closed_form():
    """r = 1, G = g: Y1 = a + w d, Y2 = a + beta w d (d = a - b), so one update gives
    max(0, (beta - 1) w d + P/g); two updates chain it. Swapping the two points or a sign
    slip changes these values."""
    a, b, g, p, w, beta = 2.0, 1.0, 4.0, 3.0, 0.5, 1.01
    A1, Ap, s = oracle.ibpg_block(np.array([[a]]), np.array([[b]]), np.array([[p]]),
                                  np.array([[g]]), w, beta, 1, 0.0)
    x1 = max(0.0, (beta - 1.0) * w * (a - b) + p / g)
    assert s == 1 and A1[0, 0] == pytest.approx(x1, rel=1e-15) and Ap[0, 0] == a
    A2, Ap2, s = oracle.ibpg_block(np.array([[a]]), np.array([[b]]), np.array([[p]]),
                                   np.array([[g]]), w, beta, 2, -1.0)
    x2 = max(0.0, (beta - 1.0) * w * (x1 - a) + p / g)
    assert s == 2 and A2[0, 0] == pytest.approx(x2, rel=1e-15) and Ap2[0, 0] == pytest.approx(x1)


def test_ibpg_without_extrapolation_is_ao_with_gradient_blocks():
    """delta_w = 0 makes w = 0, so both points are the current iterate: Algorithm 1 with
    repeated projected gradient steps (HER with beta0 = 0 and the "pgd" block solver)."""
    T, A0 = _problem(3)
    res = oracle.ibpg_solve(T, A0, 5, max_inner=7, tol=1e-2, delta_w=0.0)
    ref = oracle.her_solve(T, A0, 5, oracle.HERParams(beta0=0.0, inner="pgd", max_inner=7))
    for a, b in zip(res.factors, ref.factors):
        assert np.array_equal(a, b)


def test_ibpg_decreases_the_objective():
    T, A0 = _problem(4, dims=(20, 18, 16), r=4)
    res = oracle.ibpg_solve(T, A0, 20, max_inner=10)
    assert res.objective[-1] < 0.5 * res.f0
    assert all(w == 0.0 for w in res.weights[0])
    assert min(a.min() for a in res.factors) >= 0


def test_bro_schedule_numbers():
    """omega_k = k^(1/h) - 1 (0 before iteration 5), h = 3 grown by one every fifth increase
    of the error: 5^(1/3) - 1 = 0.70998, 11^(1/4) - 1 = 0.82116."""
    assert oracle.bro_omega(4, 3) == 0.0
    assert oracle.bro_omega(5, 3) == pytest.approx(0.7099759467, abs=1e-9)
    assert [oracle.bro_h(n) for n in (0, 4, 5, 9, 10)] == [3, 3, 4, 4, 5]
    assert oracle.bro_omega(11, oracle.bro_h(5)) == pytest.approx(0.8211602868, abs=1e-9)


def test_bro_without_extrapolation_is_algorithm_1():
    T, A0 = _problem(5)
    res = oracle.bro_solve(T, A0, 6, bro_start=100)
    ref, _, _ = oracle.ao_solve(T, A0, 6)
    for a, b in zip(res.factors, ref):
        assert np.array_equal(a, b)


def test_bro_extrapolates_without_projection():
    """The extrapolated blocks are not projected onto the nonnegative orthant (Sec. 3.3), so
    they can leave it, where HER's projected ones (eq. extproj_her) never do."""
    T, A0 = _problem(6, dims=(20, 18, 16), r=4)
    res = oracle.bro_solve(T, A0, 40)
    assert min(res.hat_min) < 0.0
    assert res.weights[:4] == [0.0] * 4 and res.weights[4] > 0.0
    f = [res.f0] + res.objective
    assert f[-1] < f[0]
