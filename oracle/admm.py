"""ADMM inner solver for one NNLS block (AO-ADMM, Sec. 2.1.2), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The block problem is min_{W >= 0} 1/2 || T_[i] - W B^T ||_F^2 with P = T_[i] B and
G = B^T B (Sec. 2, eq. def:grad). Sec. 2.1.2 solves it inexactly with a few steps of the
alternating direction method of multipliers and gives no details. The reading here is
the scaled form of ADMM on the splitting W = Z, with f(W) = 1/2 ||T_[i] - W B^T||^2 and the
nonnegativity indicator on Z:

    W_s = argmin_W f(W) + rho/2 ||W - Z_{s-1} + U_{s-1}||^2 = (P + rho (Z_{s-1} - U_{s-1})) (G + rho I)^-1
    Z_s = max(0, W_s + U_{s-1})
    U_s = U_{s-1} + W_s - Z_s

with rho = trace(G) / r (the step of the AO-ADMM method the paper cites), Z_0 the warm
start, U_0 = 0 at the start of every block solve (each block solve is then a function of
its warm start, P and G only, like the other inner solvers), and the block's iterate the
nonnegative Z_s. The inner stopping rule is the one of Sec. 4.1 (at most `max_iters`
steps, stop after step s when ||Z_s - Z_{s-1}||_F <= tol ||Z_1 - Z_0||_F). A zero G
(every component dead) gives Z = 0.
"""
from __future__ import annotations

import numpy as np


def admm_rho(G: np.ndarray) -> float:
    """rho = trace(G) / r."""
    G = np.asarray(G, dtype=np.float64)
    return float(np.trace(G)) / G.shape[0]


def admm(W0, P, G, max_iters: int = 50, tol: float = 1e-2, return_dual: bool = False):
    """ADMM steps on one block (reading above); returns (Z, steps_done, deltas[, U])."""
    Z = np.array(W0, dtype=np.float64, copy=True)
    P = np.asarray(P, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    r = G.shape[0]
    U = np.zeros_like(Z)
    rho = admm_rho(G)
    deltas = []
    if rho <= 0.0:
        Z = np.zeros_like(Z)
        return (Z, 1, [0.0], U) if return_dual else (Z, 1, [0.0])
    M = G + rho * np.eye(r)
    d1 = None
    s = 0
    for s in range(1, max_iters + 1):
        Z_prev = Z
        # W (G + rho I) = P + rho (Z - U), solved row by row (M is symmetric)
        W = np.linalg.solve(M, (P + rho * (Z - U)).T).T
        Z = np.maximum(0.0, W + U)
        U = U + W - Z
        d = float(np.linalg.norm((Z - Z_prev).ravel()))
        deltas.append(d)
        if d1 is None:
            d1 = d
            if d == 0.0:
                break
        elif d <= tol * d1:
            break
    return (Z, s, deltas, U) if return_dual else (Z, s, deltas)
