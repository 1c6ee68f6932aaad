"""Squared-error CP loss and its gradient, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss here is L = || T - [[A^(1..N)]] ||_F^2 without the paper's 1/2, so
grad_{A^(i)} L = 2 grad_{A^(i)} F with grad F from Sec. 2, eq. def:grad.
"""
from __future__ import annotations

import numpy as np

from .tensor import gradient, kruskal


def cp_loss(T: np.ndarray, factors) -> float:
    R = np.asarray(T, dtype=np.float64) - kruskal(factors)
    return float(np.sum(R * R))


def cp_loss_grad(T: np.ndarray, factors):
    """(L, [dL/dA^(1), ..., dL/dA^(N)]) with dL/dA^(i) = 2 (A^(i) B^T - T_[i]) B."""
    return cp_loss(T, factors), [2.0 * gradient(T, factors, i) for i in range(len(factors))]
