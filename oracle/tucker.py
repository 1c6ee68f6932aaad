"""Tucker-compressed NTF objective and gradient (Appendix A), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The data tensor is given in Tucker format T = (U^(1) (x) ... (x) U^(N)) G with core G of
shape (r_1, ..., r_N) and bases U^(p) of shape n_p x r_p. The objective F_t is eq.
objFunTucker; its gradient (Appendix A) only needs the small products (U^(p))^T A^(p):

  grad_{A^(i)} F_t = - U^(i) G_[i] [KR of (U^(p))^T A^(p), p != i] + A^(i) [Hadamard of the
                     other Grams],

where the Khatri-Rao product is taken in the same order as for the uncompressed MTTKRP,
so the first term is U^(i) times the MTTKRP of the core with the projected factors.
"""
from __future__ import annotations

import numpy as np

from .her import HERParams, her_solve
from .tensor import hadamard_gram, kruskal, mttkrp


def tucker_full(core: np.ndarray, bases) -> np.ndarray:
    """Expand (U^(1) (x) ... (x) U^(N)) G to a dense tensor (n-mode products)."""
    X = np.asarray(core, dtype=np.float64)
    for p, U in enumerate(bases):
        U = np.asarray(U, dtype=np.float64)
        X = np.moveaxis(np.tensordot(U, X, axes=([1], [p])), 0, p)
    return X


def tucker_mttkrp(core: np.ndarray, bases, factors, i: int) -> np.ndarray:
    """MTTKRP of the Tucker-format tensor in mode i: U^(i) [ G_[i] KR((U^(p))^T A^(p)) ]."""
    proj = [np.asarray(U, dtype=np.float64).T @ np.asarray(A, dtype=np.float64)
            for U, A in zip(bases, factors)]
    return np.asarray(bases[i], dtype=np.float64) @ mttkrp(core, proj, i)


def tucker_objective(core: np.ndarray, bases, factors) -> float:
    """F_t = 1/2 || (U (x) ...) G - [[A]] ||_F^2 from the explicit residual (eq. objFunTucker)."""
    R = tucker_full(core, bases) - kruskal(factors)
    return 0.5 * float(np.sum(R * R))


def tucker_gradient(core: np.ndarray, bases, factors, i: int) -> np.ndarray:
    """grad_{A^(i)} F_t as written in Appendix A."""
    A = np.asarray(factors[i], dtype=np.float64)
    return -tucker_mttkrp(core, bases, factors, i) + A @ hadamard_gram(factors, i)


def tucker_norm2(core: np.ndarray, bases) -> float:
    """||(U^(1) (x) ... (x) U^(N)) G||_F^2 = <G x_1 (U^(1)T U^(1)) ... x_N (U^(N)T U^(N)), G>
    (||G||^2 when every basis has orthonormal columns), without forming the tensor."""
    G = np.asarray(core, dtype=np.float64)
    X = G
    for p, U in enumerate(bases):
        U = np.asarray(U, dtype=np.float64)
        X = np.moveaxis(np.tensordot(U.T @ U, X, axes=([1], [p])), 0, p)
    return float(np.sum(X * G))


def tucker_relative_error(core: np.ndarray, bases, factors) -> float:
    """||T - [[A]]||_F / ||T||_F for Tucker-format T without forming it:
    ||T - [[A]]||^2 = ||T||^2 - 2 <G, [[(U^(1))^T A^(1), ...]]> + sum of the Hadamard product
    of all factor Grams (the cross term is the core's inner product with the Kruskal tensor
    of the projected factors, since the bases act on both sides of <T, [[A]]>)."""
    proj = [np.asarray(U, dtype=np.float64).T @ np.asarray(A, dtype=np.float64)
            for U, A in zip(bases, factors)]
    cross = float(np.sum(np.asarray(core, dtype=np.float64) * kruskal(proj)))
    H = np.ones((proj[0].shape[1],) * 2)
    for A in factors:
        A = np.asarray(A, dtype=np.float64)
        H = H * (A.T @ A)
    n2 = tucker_norm2(core, bases)
    return float(np.sqrt(max(n2 - 2.0 * cross + float(H.sum()), 0.0) / n2))


def tucker_her_solve(core: np.ndarray, bases, A0, iters: int,
                     params: HERParams = HERParams()):
    """Algorithm 2 on the Tucker-format tensor (Appendix A): the block problems and F-hat
    use the compressed MTTKRP U^(i) G_[i] KR((U^(p))^T A^(p)) and ||T||^2 of the format,
    so the full tensor is never formed."""
    return her_solve(None, A0, iters, params,
                     mttkrp_fn=lambda A, n: tucker_mttkrp(core, bases, A, n),
                     normT2=tucker_norm2(core, bases))
