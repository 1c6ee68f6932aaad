"""Tensor algebra of the NTF problem, float64, written from the paper's definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions
-----------
* A tensor is a C-order numpy array T of shape (I_1, ..., I_N) (0-based modes in code,
  1-based in the paper).
* A factor A^(i) is an I_i x r float64 matrix whose column p is a_p^(i).
"""
from __future__ import annotations

import numpy as np


def kron_columns(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Kronecker product of two column vectors (Sec. 1, Notation, eq. Kron).

    Block row j of (a kron b) is a[j] * b, so b's index runs fastest.
    """
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    out = np.empty(a.size * b.size)
    for j in range(a.size):
        out[j * b.size:(j + 1) * b.size] = a[j] * b
    return out


def khatri_rao(mats) -> np.ndarray:
    """Column-wise Kronecker product M_1 (.) M_2 (.) ... (.) M_k (Sec. 1, eq. kr).

    Column p is M_1[:, p] kron M_2[:, p] kron ... kron M_k[:, p] (associativity).
    """
    mats = [np.asarray(M, dtype=np.float64) for M in mats]
    r = mats[0].shape[1]
    for M in mats:
        if M.shape[1] != r:
            raise ValueError("Khatri-Rao factors need the same number of columns")
    cols = []
    for p in range(r):
        c = mats[0][:, p]
        for M in mats[1:]:
            c = kron_columns(c, M[:, p])
        cols.append(c)
    return np.stack(cols, axis=1)


def unfold(T: np.ndarray, i: int) -> np.ndarray:
    """Mode-i unfolding T_[i] matching the ordering of the unfolding identity (eq. unfold).

    eq. unfold writes X_[i] = A^(i) (A^(N) (.) ... (.) A^(i+1) (.) A^(i-1) (.) ... (.) A^(1))^T.
    With the Kronecker ordering of eq. Kron, the row of that Khatri-Rao product for the
    multi-index (j_l)_{l != i} is laid out with j_N slowest and j_1 fastest, so column
    c of T_[i] is the multi-index with the lowest remaining mode varying fastest.
    The paper notes other unfolding conventions exist; MTTKRP values do not depend on it
    as long as unfolding and Khatri-Rao ordering agree.
    """
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    rest = [l for l in range(N) if l != i]
    X = np.empty((T.shape[i], int(np.prod([T.shape[l] for l in rest]))))
    # Column index: j_{rest[0]} + I_{rest[0]} * (j_{rest[1]} + I_{rest[1]} * (...)).
    for idx in np.ndindex(*T.shape):
        c = 0
        for l in reversed(rest):
            c = c * T.shape[l] + idx[l]
        X[idx[i], c] = T[idx]
    return X


def _unfold_fast(T: np.ndarray, i: int) -> np.ndarray:
    """Same matrix as `unfold`, by axis permutation instead of an element loop.

    Moving mode i to the front and reading the remaining axes in Fortran order (first
    remaining mode fastest) gives the column ordering `unfold` documents.
    """
    T = np.asarray(T, dtype=np.float64)
    return np.reshape(np.moveaxis(T, i, 0), (T.shape[i], -1), order="F")


def fold(X: np.ndarray, i: int, dims) -> np.ndarray:
    """Inverse of `unfold` for a tensor of shape `dims`."""
    dims = tuple(int(d) for d in dims)
    moved = (dims[i],) + tuple(d for l, d in enumerate(dims) if l != i)
    return np.moveaxis(np.reshape(X, moved, order="F"), 0, i)


def kruskal(factors) -> np.ndarray:
    """[[A^(1), ..., A^(N)]] = sum_p a_p^(1) o ... o a_p^(N) (Sec. 1, eq. NTF, eq. kruskal)."""
    factors = [np.asarray(A, dtype=np.float64) for A in factors]
    dims = tuple(A.shape[0] for A in factors)
    r = factors[0].shape[1]
    X = np.zeros(dims)
    for p in range(r):
        term = factors[0][:, p]
        for A in factors[1:]:
            term = np.multiply.outer(term, A[:, p])
        X += term
    return X


def block_matrix(factors, i: int) -> np.ndarray:
    """B^(i) = A^(N) (.) ... (.) A^(i+1) (.) A^(i-1) (.) ... (.) A^(1) (Sec. 2, eq. def:B)."""
    N = len(factors)
    order = [l for l in range(N - 1, -1, -1) if l != i]
    return khatri_rao([factors[l] for l in order])


def mttkrp(T: np.ndarray, factors, i: int) -> np.ndarray:
    """Matricized tensor times Khatri-Rao product T_[i] B^(i) (the data term of eq. def:grad).

    factors[i] is not used. Entrywise this equals
    P[j, p] = sum over all other indices of T[..., j, ...] * prod_{l != i} A^(l)[j_l, p].
    """
    return _unfold_fast(T, i) @ block_matrix(factors, i)


def mttkrp_rows(T: np.ndarray, factors, i: int, rows) -> np.ndarray:
    """Rows `rows` of the mode-i MTTKRP, (rows of T_[i]) B^(i), without unfolding all of T.

    Row j of T_[i] is the slice of T at index j in mode i, read with the lowest remaining
    mode fastest (the column order of `unfold`).
    """
    B = block_matrix(factors, i)
    out = []
    for j in rows:
        row = np.ravel(np.take(np.asarray(T), j, axis=i), order="F").astype(np.float64)
        out.append(row @ B)
    return np.stack(out)


def gram(A: np.ndarray) -> np.ndarray:
    """A^T A (r x r)."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def hadamard_gram(factors, i: int) -> np.ndarray:
    """Hadamard product of the Grams of every factor but i (Appendix A gradient).

    Equals (B^(i))^T B^(i), the matrix of the quadratic term of eq. def:grad.
    """
    r = np.asarray(factors[0]).shape[1]
    G = np.ones((r, r))
    for l, A in enumerate(factors):
        if l != i:
            G = G * gram(A)
    return G


def objective(T: np.ndarray, factors) -> float:
    """F = 1/2 || T - [[A^(1), ..., A^(N)]] ||_F^2, formed from the explicit residual
    (Sec. 2, eq. objFun)."""
    R = np.asarray(T, dtype=np.float64) - kruskal(factors)
    return 0.5 * float(np.sum(R * R))


def gradient(T: np.ndarray, factors, i: int) -> np.ndarray:
    """grad_{A^(i)} F = (A^(i) (B^(i))^T - T_[i]) B^(i), literally (Sec. 2, eq. def:grad)."""
    B = block_matrix(factors, i)
    A = np.asarray(factors[i], dtype=np.float64)
    return (A @ B.T - _unfold_fast(T, i)) @ B
