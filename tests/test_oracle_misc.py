"""Pins for the oracle's loss/gradient, error measures, Tucker path, and the input generator."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import tucker


def test_loss_gradient_matches_fp64_central_differences_24cube():
    """FD instance of the loss workload: 24^3, r = 4; step 1e-6 * max(1, |x|)."""
    pr = synth.workload("cube24_r4")
    A = [a.copy() for a in pr.A0]
    L, grads = oracle.cp_loss_grad(pr.T, A)
    assert L == pytest.approx(2.0 * oracle.objective(pr.T, A), rel=1e-14)
    g = np.random.default_rng(0)
    for n in range(3):
        # every entry of the 24 x 4 factor
        fd = np.zeros_like(A[n])
        for idx in np.ndindex(*A[n].shape):
            h = 1e-6 * max(1.0, abs(A[n][idx]))
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[n][idx] += h
            Am[n][idx] -= h
            fd[idx] = (oracle.cp_loss(pr.T, Ap) - oracle.cp_loss(pr.T, Am)) / (2 * h)
        rel = np.linalg.norm(grads[n] - fd) / np.linalg.norm(fd)
        assert rel <= 1e-7, (n, rel)
    del g


def test_gradient_vanishes_at_planted_solution():
    g = np.random.default_rng(1)
    A = [g.random((I, 3)) for I in (5, 6, 7)]
    T = oracle.kruskal(A)
    _, grads = oracle.cp_loss_grad(T, A)
    for G in grads:
        assert np.abs(G).max() <= 1e-11 * np.abs(T).max() ** 2


def test_factor_error_invariant_to_scaling_and_joint_permutation():
    g = np.random.default_rng(2)
    A = [g.random((I, 4)) for I in (6, 7, 8)]
    perm = np.array([2, 0, 3, 1])
    B = [a[:, perm] * g.uniform(0.5, 2.0, size=4) for a in A]
    assert oracle.factor_error(A, B) <= 1e-14
    C = [b + 0.01 * g.random(b.shape) for b in B]
    assert 0 < oracle.factor_error(A, C) < 0.05


def test_relative_error_and_fit():
    g = np.random.default_rng(3)
    A = [g.random((I, 2)) for I in (4, 5, 6)]
    T = oracle.kruskal(A)
    assert oracle.relative_error(T, A) <= 1e-15 and oracle.fit(T, A) == pytest.approx(1.0)
    Z = [np.zeros_like(a) for a in A]
    assert oracle.relative_error(T, Z) == pytest.approx(1.0)


def test_tucker_mttkrp_and_gradient_match_dense_tensor():
    """Appendix A: compressed MTTKRP / gradient equal the uncompressed ones on the
    expanded tensor."""
    g = np.random.default_rng(4)
    core = g.random((3, 4, 2))
    bases = [g.random((7, 3)), g.random((6, 4)), g.random((5, 2))]
    A = [g.random((7, 3)), g.random((6, 3)), g.random((5, 3))]
    T = tucker.tucker_full(core, bases)
    assert np.allclose(T, np.einsum("abc,ia,jb,kc->ijk", core, *bases), rtol=1e-13)
    for i in range(3):
        assert np.allclose(tucker.tucker_mttkrp(core, bases, A, i), oracle.mttkrp(T, A, i),
                           rtol=1e-12)
        assert np.allclose(tucker.tucker_gradient(core, bases, A, i),
                           oracle.gradient(T, A, i), rtol=1e-11, atol=1e-11)
    assert tucker.tucker_objective(core, bases, A) == pytest.approx(oracle.objective(T, A))


# ---------------------------------------------------------------- input generator -------

def test_bf16_rounding_matches_torch():
    g = np.random.default_rng(5)
    x = np.concatenate([g.standard_normal(100000).astype(np.float32),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 0.0, -0.0,
                                  3.0e38, 1e-40], dtype=np.float32)])
    ours = synth.bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    assert np.array_equal(synth.bf16_to_f32(ours),
                          torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_correlated_factors_have_target_correlation():
    A = synth.correlated_factors(synth.generator(0), (4000,), 8, 0.9)[0]
    C = np.corrcoef(A.T)
    off = C[~np.eye(8, dtype=bool)]
    assert np.all(A >= 0)
    assert abs(off.mean() - 0.9) < 0.01


def test_noise_reaches_exact_snr_and_planted_tensor_is_kruskal():
    g = synth.generator(0)
    A = synth.uniform_factors(g, (6, 7, 8), 3)
    Tc = synth.planted_tensor(A)
    assert np.allclose(Tc, np.einsum("ip,jp,kp->ijk", *A), rtol=1e-14)
    T, sigma, _ = synth.add_noise(g, Tc, 30.0, clip=False)
    snr = 20 * np.log10(np.linalg.norm(Tc) / np.linalg.norm(T - Tc))
    assert snr == pytest.approx(30.0, abs=1e-9)


def test_problem_generation_is_deterministic():
    a = synth.make_problem((5, 6, 7), 3, snr_db=20.0, mask_frac=0.3)
    b = synth.make_problem((5, 6, 7), 3, snr_db=20.0, mask_frac=0.3)
    assert np.array_equal(a.T, b.T)
    assert all(np.array_equal(x, y) for x, y in zip(a.A0, b.A0))
    assert a.meta["n_masked"] > 0


def test_batch_specs_ranges():
    specs = synth.batch_specs(256)
    assert len(specs) == 256
    for I1, I2, I3, r in specs:
        assert 32 <= min(I1, I2, I3) and max(I1, I2, I3) <= 160 and 5 <= r <= 20


def test_tucker_norm_and_solve_match_the_dense_tensor():
    """||T||^2 of the format equals that of the expanded tensor (also for bases without
    orthonormal columns), and Algorithm 2 on the format follows Algorithm 2 on the expanded
    tensor: the same decisions and F-hat to rounding (Appendix A: only the MTTKRP changes)."""
    g = np.random.default_rng(11)
    core = g.standard_normal((4, 3, 5))
    bases = [g.standard_normal((9, 4)), g.standard_normal((7, 3)), g.standard_normal((8, 5))]
    T = tucker.tucker_full(core, bases)
    assert tucker.tucker_norm2(core, bases) == pytest.approx(float(np.sum(T * T)), rel=1e-12)
    pr = synth.make_tucker_problem((15, 12, 40), (6, 5, 7), 4, snr_db=30.0, data_seed=3)
    T = tucker.tucker_full(pr.core, pr.bases)
    assert tucker.tucker_norm2(pr.core, pr.bases) == pytest.approx(
        float(np.sum(pr.core ** 2)), rel=1e-12)  # orthonormal bases
    res_t = tucker.tucker_her_solve(pr.core, pr.bases, pr.A0, 30)
    res_d = oracle.her_solve(T, pr.A0, 30)
    assert res_t.restart == res_d.restart
    assert np.allclose(res_t.fhat, res_d.fhat, rtol=1e-9)
    assert res_t.fhat0 == pytest.approx(res_d.fhat0, rel=1e-9)
    for a, b in zip(res_t.factors, res_d.factors):
        assert np.allclose(a, b, rtol=1e-7, atol=1e-9)


def test_tucker_relative_error_matches_the_explicit_residual():
    """The compressed ||T - [[A]]|| / ||T|| equals the explicit residual of the expanded
    tensor (non-orthonormal bases, 4-way), and is 0 at the planted factors without noise."""
    g = np.random.default_rng(12)
    core = g.standard_normal((3, 4, 2, 3))
    bases = [g.standard_normal((6, 3)), g.standard_normal((5, 4)), g.standard_normal((7, 2)),
             g.standard_normal((4, 3))]
    A = [g.random((U.shape[0], 3)) for U in bases]
    T = tucker.tucker_full(core, bases)
    ref = np.linalg.norm((T - oracle.kruskal(A)).ravel()) / np.linalg.norm(T.ravel())
    assert tucker.tucker_relative_error(core, bases, A) == pytest.approx(ref, rel=1e-12)
    pr = synth.make_tucker_problem((15, 12, 40), (6, 5, 7), 4, snr_db=None, data_seed=5)
    assert tucker.tucker_relative_error(pr.core, pr.bases, pr.A_true) < 1e-6


def test_tucker_generator_plants_the_factors_in_the_bases():
    """The bases span the planted factors, so the noiseless format is exactly [[A]]."""
    pr = synth.make_tucker_problem((15, 12, 40), (6, 5, 7), 4, snr_db=None, data_seed=5)
    for U, A in zip(pr.bases, pr.A_true):
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
        assert np.allclose(U @ (U.T @ A), A, atol=1e-12)
    assert np.allclose(tucker.tucker_full(pr.core, pr.bases), oracle.kruskal(pr.A_true),
                       atol=1e-12)
