"""Projected-gradient inner solvers for one NNLS block, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The block problem is min_{W >= 0} 1/2 || T_[i] - W B^T ||_F^2, whose gradient in W is
W G - P with P = T_[i] B and G = B^T B (Sec. 2, eq. def:grad). Restricted to the block
the objective is L-smooth with L = ||G||_2, the largest eigenvalue of the symmetric
positive semidefinite G (Sec. 2.2). Minimising its quadratic majorisation at W gives the
projected gradient step (Sec. 2.2; the step inside APG's update of Sec. 2.2.1 without
its extrapolation):

    W <- max(0, W - (W G - P) / L).

`pgd` repeats that step; `nesterov` adds Nesterov-type acceleration (Sec. 2.2 mentions
it without details; the reading here is the classical accelerated projected gradient
with t_0 = 1, t_s = (1 + sqrt(1 + 4 t_{s-1}^2)) / 2, the gradient step taken at
Y = W_s + ((t_{s-1} - 1) / t_s) (W_s - W_{s-1})). Both use the inner stopping rule the
A-HALS solver uses (Sec. 4.1): at most `max_iters` steps, stop after step s when
||W_s - W_{s-1}||_F <= tol * ||W_1 - W_0||_F. Sec. 3.1.4 runs HER with 50 such steps
(HER-PGD50, HER-Nesterov50). G = 0 (every component dead) gives W = 0.
"""
from __future__ import annotations

import numpy as np


def lipschitz(G: np.ndarray) -> float:
    """L = ||G||_2 = largest eigenvalue of the symmetric PSD matrix G (Sec. 2.2)."""
    G = np.asarray(G, dtype=np.float64)
    return float(np.linalg.eigvalsh(0.5 * (G + G.T))[-1])


def pg_step(W: np.ndarray, P: np.ndarray, G: np.ndarray, L: float) -> np.ndarray:
    """One projected gradient step max(0, W - (W G - P) / L)."""
    if L <= 0.0:
        return np.zeros_like(W)
    return np.maximum(0.0, W - (W @ G - P) / L)


def _run(W0, P, G, max_iters, tol, accelerated):
    W = np.array(W0, dtype=np.float64, copy=True)
    P = np.asarray(P, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    L = lipschitz(G)
    Y = W.copy()
    t = 1.0
    deltas = []
    d1 = None
    s = 0
    for s in range(1, max_iters + 1):
        W_prev = W
        W = pg_step(Y if accelerated else W, P, G, L)
        d = float(np.linalg.norm((W - W_prev).ravel()))
        deltas.append(d)
        if accelerated:
            t_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            Y = W + ((t - 1.0) / t_next) * (W - W_prev)
            t = t_next
        if d1 is None:
            d1 = d
            if d == 0.0:
                break
        elif d <= tol * d1:
            break
    return W, s, deltas


def pgd(W0, P, G, max_iters: int = 50, tol: float = 1e-2):
    """Repeated projected gradient steps; returns (W, steps_done, deltas)."""
    return _run(W0, P, G, max_iters, tol, accelerated=False)


def nesterov(W0, P, G, max_iters: int = 50, tol: float = 1e-2):
    """Accelerated projected gradient (reading above); returns (W, steps_done, deltas)."""
    return _run(W0, P, G, max_iters, tol, accelerated=True)
