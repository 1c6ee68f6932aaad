"""A-HALS inner solver for one NNLS block, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The block problem is min_{W >= 0} 1/2 || T_[i] - W B^T ||_F^2 with B = B^(i). Its data
enter only through P = T_[i] B (the MTTKRP) and G = B^T B (the Hadamard of the other
factors' Grams), so the solver takes (W0, P, G).

Reading of the A-HALS column update as printed (Sec. 2.1.4): the paper sets M to the
unfolding of the data tensor and H to the Khatri-Rao product, and writes rows of H where
columns are meant. With H := B^T the printed quantities are M H_{j,:}^T = P[:, j],
H_{l,:} H_{j,:}^T = G[l, j] and ||H_{j,:}||^2 = G[j, j], which gives the update below.
"""
from __future__ import annotations

import numpy as np


def hals_column(W: np.ndarray, P: np.ndarray, G: np.ndarray, j: int) -> None:
    """Exact NNLS update of column j with the other columns fixed, in place (Sec. 2.1.4).

    W[:, j] = max(0, P[:, j] - sum_{l != j} W[:, l] G[l, j]) / G[j, j].

    G[j, j] = 0 means component j is zero in some other factor; then P[:, j] and every
    G[l, j] vanish too, the column does not enter the objective, and it is set to 0
    (a dead component stays dead).
    """
    r = W.shape[1]
    others = [l for l in range(r) if l != j]
    if G[j, j] == 0.0:
        W[:, j] = 0.0
        return
    s = W[:, others] @ G[others, j] if others else np.zeros(W.shape[0])
    W[:, j] = np.maximum(0.0, P[:, j] - s) / G[j, j]


def hals(W0: np.ndarray, P: np.ndarray, G: np.ndarray, max_sweeps: int = 50,
         tol: float = 1e-2):
    """Repeated cyclic column sweeps j = 1..r (Sec. 2.1.4), with the inner stopping rule of
    Sec. 4.1: stop after `max_sweeps` sweeps, or after sweep s when
    ||W_s - W_{s-1}||_F <= tol * ||W_1 - W_0||_F (Frobenius norm; checked after every
    sweep, so sweep 1 stops only if it changed nothing). tol = 0 runs the sweeps until
    one changes nothing or `max_sweeps` is reached.

    Returns (W, sweeps_done, deltas) where deltas[s-1] = ||W_s - W_{s-1}||_F.
    """
    W = np.array(W0, dtype=np.float64, copy=True)
    P = np.asarray(P, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    r = W.shape[1]
    deltas = []
    d1 = None
    s = 0
    for s in range(1, max_sweeps + 1):
        W_prev = W.copy()
        for j in range(r):
            hals_column(W, P, G, j)
        d = float(np.linalg.norm((W - W_prev).ravel()))
        deltas.append(d)
        if d1 is None:
            d1 = d
        if d <= tol * d1:
            break
    return W, s, deltas
