"""Pins for the oracle's HER loop (Algorithm 2) and plain AO (Algorithm 1).

* The beta / beta_bar schedule against a sequence worked out by hand from eqs.
  HER_eq:beta_update and HER_eq:beta_bar_update with the default parameters.
* A full rank-one HER iteration against closed forms (for r = 1 each block problem is a
  one-variable projected least-squares fit), which pins which blocks enter each update.
* F-hat against its definition F(A-hat^(1..N-1), A^(N)) evaluated from the residual.
* beta0 = 0 reduces HER to Algorithm 1 exactly, with monotone objective (Sec. 2.1).
* Nonnegativity of every iterate (Sec. 3.1.2), exact recovery of noiseless planted data
  (Sec. 4.1: f_min = 0 when sigma = 0), resume equivalence.
"""
import numpy as np
import pytest

import oracle
import synth

P_DEF = oracle.HERParams()


def test_beta_schedule_hand_worked_sequence():
    # beta0 = 0.5, beta_bar0 = 1, gamma = 1.05, gamma_bar = 1.01, eta = 1.5.
    # accept: beta = min(beta_bar_old, 1.05 beta); beta_bar = min(1, 1.01 beta_bar_old)
    # restart: beta_bar = beta_old; beta = beta_old / 1.5
    decisions = ["a", "a", "r", "a", "r", "r", "a"]
    want_beta = [0.525, 0.55125, 0.3675, 0.385875, 0.25725, 0.1715, 0.180075]
    want_bar = [1.0, 1.0, 0.55125, 0.5567625, 0.385875, 0.25725, 0.2598225]
    b, bb = 0.5, 1.0
    for d, wb, wbb in zip(decisions, want_beta, want_bar):
        b, bb = oracle.update_beta(b, bb, d == "r", P_DEF)
        assert b == pytest.approx(wb, rel=1e-14)
        assert bb == pytest.approx(wbb, rel=1e-14)


def test_beta_capped_by_beta_bar_after_many_accepts():
    # 14 accepts: beta = 0.5 * 1.05^14 = 0.98996...; the 15th is capped at beta_bar = 1.
    b, bb = 0.5, 1.0
    for _ in range(14):
        b, bb = oracle.update_beta(b, bb, False, P_DEF)
    assert b == pytest.approx(0.5 * 1.05 ** 14, rel=1e-13) and bb == 1.0
    b, bb = oracle.update_beta(b, bb, False, P_DEF)
    assert b == 1.0 and bb == 1.0


def test_beta_invariant_over_random_decisions():
    g = np.random.default_rng(0)
    b, bb = 0.5, 1.0
    for _ in range(2000):
        b, bb = oracle.update_beta(b, bb, bool(g.random() < 0.4), P_DEF)
        assert 0.0 < b <= bb <= 1.0


def test_extrapolate_closed_form_and_projection():
    g = np.random.default_rng(1)
    new, old = g.random((5, 3)), g.random((5, 3))
    out = oracle.extrapolate(new, old, 0.7)
    for idx in np.ndindex(*new.shape):
        assert out[idx] == max(0.0, new[idx] + 0.7 * (new[idx] - old[idx]))
    assert np.all(out >= 0)


def _ttv(T, vecs, skip):
    """Contract T with a vector in every mode but `skip` (rank-one MTTKRP)."""
    X = T
    for l in reversed(range(T.ndim)):
        if l != skip:
            X = np.tensordot(X, vecs[l], axes=([l], [0]))
    return X


def test_rank_one_her_iteration_closed_form():
    g = np.random.default_rng(2)
    dims = (4, 5, 6)
    T = g.random(dims)
    a0 = [g.random(I) for I in dims]
    beta = P_DEF.beta0
    a = [v.copy() for v in a0]
    ahat = [v.copy() for v in a0]
    fhat_prev = oracle.objective(T, [v[:, None] for v in a0])
    seen = []

    def hook(k, A_prev, A_new, A_hat, fh):
        seen.append(([x.copy() for x in A_new], [x.copy() for x in A_hat], fh))

    res = oracle.her_solve(T, [v[:, None] for v in a0], iters=3, hook=hook)
    b, bb = P_DEF.beta0, 1.0
    for k in range(3):
        new = [None] * 3
        for n in range(3):
            # one-variable problem per entry: a_n = max(0, T x_{l != n} ahat_l / prod ||ahat_l||^2)
            num = _ttv(T, ahat, n)
            den = np.prod([ahat[l] @ ahat[l] for l in range(3) if l != n])
            new[n] = np.maximum(0.0, num / den)
            ahat[n] = np.maximum(0.0, new[n] + b * (new[n] - a[n]))
        fh = 0.5 * np.sum((T - np.einsum("i,j,k->ijk", ahat[0], ahat[1], new[2])) ** 2)
        got_new, got_hat, got_fh = seen[k]
        for n in range(3):
            assert np.allclose(got_new[n][:, 0], new[n], rtol=1e-12)
            assert np.allclose(got_hat[n][:, 0], ahat[n], rtol=1e-12)
        assert got_fh == pytest.approx(fh, rel=1e-10)
        restart = fh > fhat_prev
        assert res.restart[k] == restart
        if restart:
            ahat = [v.copy() for v in new]
            b, bb = b / 1.5, b
        else:
            new = [v.copy() for v in ahat]
            b, bb = min(bb, 1.05 * b), min(1.0, 1.01 * bb)
        a = new
        fhat_prev = fh
        assert res.beta[k] == pytest.approx(b) and res.beta_bar[k] == pytest.approx(bb)


def _small_problem(seed=0, dims=(12, 10, 8), r=3, snr=30.0):
    return synth.make_problem(dims, r, snr_db=snr, data_seed=seed, init_seed=seed + 100)


def test_fhat_is_objective_at_extrapolated_blocks_and_last_block():
    pr = _small_problem()
    checks = []

    def hook(k, A_prev, A_new, A_hat, fh):
        args = list(A_hat[:-1]) + [A_new[-1]]
        checks.append((fh, oracle.objective(pr.T, args)))

    res = oracle.her_solve(pr.T, pr.A0, iters=8, hook=hook)
    assert res.fhat0 == pytest.approx(oracle.objective(pr.T, pr.A0), rel=1e-12)
    for fh, ref in checks:
        assert fh == pytest.approx(ref, rel=1e-9)
    # restart flag <=> F-hat increased w.r.t. the previous iteration's F-hat
    prev = res.fhat0
    for fh, rs in zip(res.fhat, res.restart):
        assert rs == (fh > prev)
        prev = fh


def test_all_iterates_nonnegative():
    pr = _small_problem(seed=1)
    bad = []

    def hook(k, A_prev, A_new, A_hat, fh):
        for X in list(A_new) + list(A_hat):
            if np.any(X < 0):
                bad.append(k)

    oracle.her_solve(pr.T, pr.A0, iters=15, hook=hook)
    assert not bad


def test_beta0_zero_is_plain_ao_with_monotone_objective():
    pr = _small_problem(seed=2, dims=(9, 8, 7, 6), r=3)
    p0 = oracle.HERParams(beta0=0.0)
    res = oracle.her_solve(pr.T, pr.A0, iters=12, params=p0)
    A_ao, objs, sweeps = oracle.ao_solve(pr.T, pr.A0, iters=12, record_objective=True)
    for x, y in zip(res.factors, A_ao):
        assert np.array_equal(x, y)
    assert res.sweeps == sweeps
    assert all(b == 0.0 for b in res.beta)
    for fh, f in zip(res.fhat, objs):
        assert fh == pytest.approx(f, rel=1e-9)
    for a, b in zip(objs, objs[1:]):
        assert b <= a * (1 + 1e-12)


def test_resume_matches_uninterrupted_run():
    pr = _small_problem(seed=3)
    full = oracle.her_solve(pr.T, pr.A0, iters=10)
    first = oracle.her_solve(pr.T, pr.A0, iters=4)
    rest = oracle.her_solve(pr.T, None, iters=6, state=first.state)
    for x, y in zip(full.factors, rest.factors):
        assert np.array_equal(x, y)
    assert full.fhat == first.fhat + rest.fhat
    assert full.restart == first.restart + rest.restart


@pytest.mark.slow
def test_exact_recovery_noiseless_planted_cube():
    """Noiseless planted 50^3, r = 10 (the first synthetic shape of Sec. 4): f_min = 0."""
    pr = synth.make_problem((50, 50, 50), 10, snr_db=None, data_seed=0, init_seed=1)
    res = oracle.her_solve(pr.T, pr.A0, iters=300)
    assert oracle.relative_error(pr.T, res.factors) <= 1e-6
    assert oracle.factor_error(pr.A_true, res.factors) <= 1e-4


@pytest.mark.slow
def test_her_not_worse_than_plain_ahals_on_small_cube():
    """Direction of the paper's main claim (Sec. 4): after the same number of outer
    iterations HER-A-HALS reaches an objective no larger than A-HALS."""
    pr = synth.workload("cube50_r10")
    her = oracle.her_solve(pr.T, pr.A0, iters=100)
    A_ao, _, _ = oracle.ao_solve(pr.T, pr.A0, iters=100)
    assert oracle.objective(pr.T, her.factors) <= oracle.objective(pr.T, A_ao)


def test_equal_fhat_accepts_zero_tensor():
    """T = 0: every block collapses to 0 (dead components), F-hat_k = 0 for all k >= 1, so
    from k = 2 on F-hat ties with the previous value; a tie accepts (strict '>' restarts)."""
    g = np.random.default_rng(5)
    dims = (4, 5, 6)
    A0 = [g.random((I, 2)) for I in dims]
    res = oracle.her_solve(np.zeros(dims), A0, iters=3)
    assert res.fhat == [0.0, 0.0, 0.0]
    assert res.restart == [False, False, False]
    assert res.beta == pytest.approx([0.525, 0.55125, 0.5788125])
    assert all(np.all(f == 0.0) for f in res.factors)
