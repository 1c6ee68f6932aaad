"""Error measures of the experiments section, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment

from .tensor import kruskal


def residual_norm(T: np.ndarray, factors) -> float:
    """|| T - [[A]] ||_F from the explicit residual (data-fitting error, eq. err_true_def,
    without the 1/2 and the square)."""
    R = np.asarray(T, dtype=np.float64) - kruskal(factors)
    return float(np.sqrt(np.sum(R * R)))


def relative_error(T: np.ndarray, factors) -> float:
    """|| T - [[A]] ||_F / || T ||_F."""
    T = np.asarray(T, dtype=np.float64)
    return residual_norm(T, factors) / float(np.sqrt(np.sum(T * T)))


def fit(T: np.ndarray, factors) -> float:
    """1 - relative error."""
    return 1.0 - relative_error(T, factors)


def _normalize_columns(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    n = np.linalg.norm(A, axis=0)
    n = np.where(n == 0.0, 1.0, n)
    return A / n


def factor_error(A_true, A) -> float:
    """Factor-fitting error e (Sec. 4.1, eq. err_fact_def).

    Columns are normalized to unit 2-norm; one column permutation, found with the
    Hungarian algorithm, matches the estimate to the truth. The paper writes the
    permutation inside the sum over modes; since CP components permute jointly across
    modes, one permutation is shared by all modes, chosen on the summed squared
    distances.
    """
    N = len(A_true)
    r = np.asarray(A_true[0]).shape[1]
    Xt = [_normalize_columns(a) for a in A_true]
    Xe = [_normalize_columns(a) for a in A]
    cost = np.zeros((r, r))
    for n in range(N):
        # cost[p, q] = || true col p - estimated col q ||^2 summed over modes
        diff = Xt[n][:, :, None] - Xe[n][:, None, :]
        cost += np.sum(diff * diff, axis=0)
    rows, cols = linear_sum_assignment(cost)
    perm = np.empty(r, dtype=int)
    perm[rows] = cols
    e = 0.0
    for n in range(N):
        e += np.linalg.norm(Xt[n] - Xe[n][:, perm]) / np.linalg.norm(Xt[n])
    return e / N
