"""Pins for the oracle's tensor algebra (MTTKRP, unfolding, Grams, objective, gradient).

Each test checks the oracle against something other than itself: element loops written
from the entrywise definition, numpy.einsum / numpy.kron / a plain matrix product, closed
forms of rank-one tensors, or identities between independently computed quantities.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.tensor import _unfold_fast

SHAPES = [(3, 4, 5), (2, 3, 4, 5), (4, 1, 3), (5, 6)]


def _rand_factors(g, dims, r):
    return [g.random((I, r)) for I in dims]


def _mttkrp_loops(T, factors, i):
    """Entrywise definition: P[j,p] = sum over the other indices of T * prod of factors."""
    dims = T.shape
    r = factors[0].shape[1]
    P = np.zeros((dims[i], r))
    for idx in itertools.product(*[range(d) for d in dims]):
        for p in range(r):
            w = T[idx]
            for l, A in enumerate(factors):
                if l != i:
                    w *= A[idx[l], p]
            P[idx[i], p] += w
    return P


def _einsum_mttkrp(T, factors, i):
    letters = "abcdefgh"[:T.ndim]
    ins = [letters] + [letters[l] + "z" for l in range(T.ndim) if l != i]
    ops = [T] + [factors[l] for l in range(T.ndim) if l != i]
    return np.einsum(",".join(ins) + "->" + letters[i] + "z", *ops)


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_mttkrp_matches_entrywise_loops_and_einsum(dims, r):
    g = np.random.default_rng(7)
    T = g.standard_normal(dims)
    A = _rand_factors(g, dims, r)
    for i in range(len(dims)):
        P = oracle.mttkrp(T, A, i)
        ref = _mttkrp_loops(T, A, i)
        assert np.allclose(P, ref, rtol=1e-13, atol=1e-13)
        assert np.allclose(P, _einsum_mttkrp(T, A, i), rtol=1e-13, atol=1e-13)


def test_mttkrp_ignores_own_factor():
    g = np.random.default_rng(1)
    T = g.random((3, 4, 5))
    A = _rand_factors(g, T.shape, 3)
    B = [a.copy() for a in A]
    B[1] = g.random(B[1].shape) * 100
    assert np.array_equal(oracle.mttkrp(T, A, 1), oracle.mttkrp(T, B, 1))


def test_mttkrp_rank_one_closed_form():
    """T = a o b o c and factors (., b, c): P_1 = a ||b||^2 ||c||^2 (and cyclically)."""
    g = np.random.default_rng(3)
    a, b, c = g.random(4), g.random(5), g.random(6)
    T = np.multiply.outer(np.multiply.outer(a, b), c)
    F = [a[:, None], b[:, None], c[:, None]]
    assert np.allclose(oracle.mttkrp(T, F, 0)[:, 0], a * (b @ b) * (c @ c), rtol=1e-14)
    assert np.allclose(oracle.mttkrp(T, F, 1)[:, 0], b * (a @ a) * (c @ c), rtol=1e-14)
    assert np.allclose(oracle.mttkrp(T, F, 2)[:, 0], c * (a @ a) * (b @ b), rtol=1e-14)


def test_mttkrp_matrix_case_is_a_matrix_product():
    """N = 2 is NMF (Sec. 1): P_1 = T A^(2), P_2 = T^T A^(1)."""
    g = np.random.default_rng(4)
    T = g.random((7, 9))
    A = _rand_factors(g, T.shape, 3)
    assert np.allclose(oracle.mttkrp(T, A, 0), T @ A[1], rtol=1e-14)
    assert np.allclose(oracle.mttkrp(T, A, 1), T.T @ A[0], rtol=1e-14)


@pytest.mark.parametrize("dims", SHAPES[:2])
def test_mttkrp_cross_mode_inner_product(dims):
    """<P_n, A^(n)> = <T, [[A]]> for every mode n."""
    g = np.random.default_rng(5)
    T = g.random(dims)
    A = _rand_factors(g, dims, 3)
    ref = float(np.sum(T * oracle.kruskal(A)))
    for n in range(len(dims)):
        assert np.isclose(np.sum(oracle.mttkrp(T, A, n) * A[n]), ref, rtol=1e-13)


@pytest.mark.parametrize("dims", SHAPES)
def test_unfold_fast_matches_element_loop_and_fold(dims):
    T = np.random.default_rng(2).random(dims)
    for i in range(len(dims)):
        X = oracle.unfold(T, i)
        assert np.array_equal(X, _unfold_fast(T, i))
        assert np.array_equal(oracle.fold(X, i, dims), T)


@pytest.mark.parametrize("dims", SHAPES[:2])
def test_unfolding_identity_of_kruskal_tensor(dims):
    """eq. unfold: X_[i] = A^(i) B^(i)^T for X = [[A]] built from outer products."""
    g = np.random.default_rng(6)
    A = _rand_factors(g, dims, 3)
    X = oracle.kruskal(A)
    for i in range(len(dims)):
        assert np.allclose(oracle.unfold(X, i), A[i] @ oracle.block_matrix(A, i).T, rtol=1e-13)


def test_khatri_rao_is_columnwise_numpy_kron():
    g = np.random.default_rng(8)
    M = [g.random((3, 4)), g.random((2, 4)), g.random((5, 4))]
    K = oracle.khatri_rao(M)
    for p in range(4):
        assert np.allclose(K[:, p], np.kron(np.kron(M[0][:, p], M[1][:, p]), M[2][:, p]))


def test_kruskal_matches_einsum():
    g = np.random.default_rng(9)
    A = _rand_factors(g, (3, 4, 5), 2)
    assert np.allclose(oracle.kruskal(A), np.einsum("ip,jp,kp->ijk", *A), rtol=1e-14)


@pytest.mark.parametrize("dims", SHAPES[:2])
def test_hadamard_of_grams_equals_block_gram(dims):
    """(B^(i))^T B^(i) from the explicit Khatri-Rao matrix = Hadamard of the other Grams."""
    g = np.random.default_rng(10)
    A = _rand_factors(g, dims, 4)
    for i in range(len(dims)):
        B = oracle.block_matrix(A, i)
        assert np.allclose(B.T @ B, oracle.hadamard_gram(A, i), rtol=1e-13)


def test_kruskal_norm_from_grams():
    """||[[A]]||^2 = 1^T (Hadamard of all Grams) 1."""
    g = np.random.default_rng(11)
    A = _rand_factors(g, (4, 5, 6), 3)
    G = np.ones((3, 3))
    for a in A:
        G = G * (a.T @ a)
    assert np.isclose(np.sum(oracle.kruskal(A) ** 2), G.sum(), rtol=1e-13)


def test_objective_zero_on_planted_and_matches_gram_trick():
    g = np.random.default_rng(12)
    A = _rand_factors(g, (6, 7, 8), 3)
    T = oracle.kruskal(A)
    assert oracle.objective(T, A) <= 1e-24 * np.sum(T * T)
    T2 = T + 0.1 * g.standard_normal(T.shape)
    B = _rand_factors(g, T.shape, 3)
    N = 3
    P = oracle.mttkrp(T2, B, N - 1)
    G = oracle.hadamard_gram(B, N - 1)
    fh = oracle.f_hat(np.sum(T2 * T2), P, B[N - 1], G)
    assert np.isclose(fh, oracle.objective(T2, B), rtol=1e-12)


def test_gradient_matches_central_differences_and_gram_form():
    g = np.random.default_rng(13)
    dims = (4, 5, 3)
    T = g.random(dims)
    A = _rand_factors(g, dims, 2)
    for i in range(3):
        grad = oracle.gradient(T, A, i)
        alt = A[i] @ oracle.hadamard_gram(A, i) - oracle.mttkrp(T, A, i)
        assert np.allclose(grad, alt, rtol=1e-12, atol=1e-12)
        fd = np.zeros_like(A[i])
        for idx in np.ndindex(*A[i].shape):
            h = 1e-6
            Ap = [a.copy() for a in A]
            Am = [a.copy() for a in A]
            Ap[i][idx] += h
            Am[i][idx] -= h
            fd[idx] = (oracle.objective(T, Ap) - oracle.objective(T, Am)) / (2 * h)
        assert np.allclose(grad, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("dims", SHAPES)
def test_mttkrp_rows_match_full_mttkrp(dims):
    g = np.random.default_rng(14)
    T = g.random(dims)
    A = _rand_factors(g, dims, 3)
    for i in range(len(dims)):
        P = _mttkrp_loops(T, A, i)
        rows = list(range(dims[i]))
        assert np.allclose(oracle.mttkrp_rows(T, A, i, rows), P, rtol=1e-13, atol=1e-13)
