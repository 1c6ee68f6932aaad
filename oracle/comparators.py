"""The paper's comparison algorithms on the same block problems, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* APG (Sec. 2.2.1; pseudocode: Appendix, algorithm APG): per outer iteration k and block
  i, an extrapolation point inside the block update followed by one projected gradient
  step, and a restart that redoes the whole iteration without extrapolation when the
  objective increased.
* iBPG (Sec. 2.2.2; Appendix, algorithm iBPG): two extrapolation points (one for the
  gradient, one for the inertia), several updates per block, no restart.
* Bro's extrapolation in the modified, block-wise form of Sec. 3.3 ("The modified
  implementation of Bro, GR and LS"): Algorithm 2's structure (each block extrapolated
  right after its update, the extrapolated sequence abandoned when the error increases),
  with HER's beta replaced by omega_k = k^(1/h(k)) - 1 and no projection of the
  extrapolated point (the scheme is not modified for nonnegativity).

Readings of points the paper leaves open (each one a single place below):
* t_k (APG, iBPG) depends only on k: the same t_k serves every block of iteration k.
* L^(i)_{k-1} = ||G||_2 of block i's problem at iteration k (G = B^T B built from the
  other blocks' current values); at k = 1 the ratio L_{k-2} / L_{k-1} is taken as 1 (the
  first weight w_0 = (t_0 - 1) / t_1 = 0 anyway).
* The second initial point A_{-1} of both methods is A_0.
* APG's delta_w ("choose delta_w < 1") is 0.9999; iBPG's delta_w = 0.99 and beta = 1.01
  are the pseudocode's values.
* APG's restart redoes every block in order, each with the other blocks' latest values
  (a plain block projected-gradient sweep from A_{k-1}); t_k is not reset.
* iBPG's inner "until some criteria": at most `max_inner` updates with the inner stopping
  rule of Sec. 4.1 on ||A_cur - A_prev||; the weight w is fixed for the block's updates.
* Bro: omega_k = 0 for k < `bro_start` (= 5: "no extrapolation in the first few
  iterations"); h(1) = 3, and h grows by one each time the error has increased in more
  than four iterations since it last grew (every fifth restart).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .hals import hals
from .her import f_hat
from .pgd import lipschitz, pg_step
from .tensor import hadamard_gram, mttkrp, objective


def t_next(t: float) -> float:
    """t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2."""
    return 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))


def _weight(w_hat: float, delta_w: float, L_prev, L_cur: float) -> float:
    """w = min(w_hat, delta_w sqrt(L_{k-2} / L_{k-1})) (ratio 1 without a previous L)."""
    ratio = 1.0 if (L_prev is None or L_cur <= 0.0) else L_prev / L_cur
    return min(w_hat, delta_w * float(np.sqrt(ratio)))


@dataclass
class CompResult:
    factors: list
    objective: list = field(default_factory=list)  # F(A_k) after each iteration
    restart: list = field(default_factory=list)    # APG / Bro: True if iteration k restarted
    weights: list = field(default_factory=list)    # per iteration: w (APG, iBPG) or omega
    history: list = field(default_factory=list)    # keep_history: factors after each iteration
    hat_min: list = field(default_factory=list)    # Bro: smallest entry of the extrapolated blocks
    f0: float = 0.0


def apg_solve(T: np.ndarray, A0, iters: int, delta_w: float = 0.9999,
              keep_history: bool = False) -> CompResult:
    """APG for `iters` outer iterations (readings above)."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    normT2 = float(np.sum(T * T))
    A_prev = [np.array(a, dtype=np.float64, copy=True) for a in A0]  # A_{k-2}
    A = [a.copy() for a in A_prev]                                     # A_{k-1}
    L_prev = [None] * N
    t = 1.0
    f_prev = objective(T, A)
    res = CompResult(factors=[], f0=f_prev)
    for _k in range(iters):
        tn = t_next(t)
        w_hat = (t - 1.0) / tn
        A_new = [a.copy() for a in A]
        L_cur, ws = [0.0] * N, []
        P = G = None
        for i in range(N):
            G = hadamard_gram(A_new, i)   # blocks < i: this iteration's; > i: A_{k-1}
            P = mttkrp(T, A_new, i)
            L_cur[i] = lipschitz(G)
            w = _weight(w_hat, delta_w, L_prev[i], L_cur[i])
            ws.append(w)
            A_hat = A[i] + w * (A[i] - A_prev[i])
            A_new[i] = pg_step(A_hat, P, G, L_cur[i])
        f = f_hat(normT2, P, A_new[N - 1], G)
        restart = f > f_prev
        if restart:
            # redo the iteration with the unextrapolated points A_{k-1}
            A_new = [a.copy() for a in A]
            for i in range(N):
                G = hadamard_gram(A_new, i)
                P = mttkrp(T, A_new, i)
                L_cur[i] = lipschitz(G)
                A_new[i] = pg_step(A[i], P, G, L_cur[i])
            f = f_hat(normT2, P, A_new[N - 1], G)
        A_prev, A = A, A_new
        L_prev = L_cur
        t = tn
        f_prev = f
        res.objective.append(f)
        res.restart.append(bool(restart))
        res.weights.append(ws)
        if keep_history:
            res.history.append([a.copy() for a in A])
    res.factors = A
    return res


def ibpg_block(A_cur, A_prv, P, G, w: float, beta: float, max_inner: int, tol: float):
    """iBPG's updates of one block with w fixed: Y1 = A_cur + w (A_cur - A_prev) (gradient
    point), Y2 = A_cur + beta w (A_cur - A_prev) (inertial point), A_prev <- A_cur,
    A_cur <- max(0, Y2 - (Y1 G - P) / L), L = ||G||_2, with the inner stopping rule.
    Returns (A_cur, A_prev, updates done)."""
    A_cur = np.array(A_cur, dtype=np.float64, copy=True)
    A_prv = np.array(A_prv, dtype=np.float64, copy=True)
    P = np.asarray(P, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    L = lipschitz(G)
    d1 = None
    s = 0
    for s in range(1, max_inner + 1):
        diff = A_cur - A_prv
        Y1 = A_cur + w * diff
        Y2 = A_cur + beta * w * diff
        A_prv = A_cur
        A_cur = np.maximum(0.0, Y2 - (Y1 @ G - P) / L) if L > 0.0 else np.zeros_like(A_cur)
        d = float(np.linalg.norm((A_cur - A_prv).ravel()))
        if d1 is None:
            d1 = d
            if d == 0.0:
                break
        elif d <= tol * d1:
            break
    return A_cur, A_prv, s


def ibpg_solve(T: np.ndarray, A0, iters: int, max_inner: int = 50, tol: float = 1e-2,
               delta_w: float = 0.99, beta: float = 1.01) -> CompResult:
    """iBPG for `iters` outer iterations (readings above)."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    normT2 = float(np.sum(T * T))
    A_cur = [np.array(a, dtype=np.float64, copy=True) for a in A0]
    A_prv = [a.copy() for a in A_cur]  # A_{-1} = A_0
    L_prev = [None] * N
    t = 1.0
    res = CompResult(factors=[], f0=objective(T, A_cur))
    for _k in range(iters):
        tn = t_next(t)
        w_hat = (t - 1.0) / tn
        ws = []
        L_cur = [0.0] * N
        P = G = None
        for i in range(N):
            G = hadamard_gram(A_cur, i)
            P = mttkrp(T, A_cur, i)
            L_cur[i] = lipschitz(G)
            w = _weight(w_hat, delta_w, L_prev[i], L_cur[i])
            ws.append(w)
            A_cur[i], A_prv[i], _ = ibpg_block(A_cur[i], A_prv[i], P, G, w, beta, max_inner,
                                               tol)
        L_prev = L_cur
        t = tn
        res.objective.append(f_hat(normT2, P, A_cur[N - 1], G))
        res.weights.append(ws)
    res.factors = A_cur
    return res


def bro_h(nrestarts: int) -> int:
    """h after `nrestarts` increases of the error: 3, grown by one every fifth increase."""
    return 3 + nrestarts // 5


def bro_omega(k: int, h: int, bro_start: int = 5) -> float:
    """omega_k = k^(1/h) - 1, and 0 for k < bro_start."""
    return 0.0 if k < bro_start else float(k) ** (1.0 / h) - 1.0


def bro_solve(T: np.ndarray, A0, iters: int, max_inner: int = 50, tol: float = 1e-2,
              bro_start: int = 5) -> CompResult:
    """Bro's extrapolation in the block-wise HER structure with A-HALS blocks (Bro-AHALS of
    Sec. 3.3 and Sec. 4): iteration k updates block n from the extrapolated blocks of this
    iteration (l < n) and of the previous one (l > n), then extrapolates it by omega_k
    without projection; F-hat_k as in Algorithm 2 decides whether the extrapolated sequence
    is kept."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    normT2 = float(np.sum(T * T))
    A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
    A_hat = [a.copy() for a in A]
    f_prev = objective(T, A)
    nrestarts = 0
    res = CompResult(factors=[], f0=f_prev)
    for k in range(1, iters + 1):
        omega = bro_omega(k, bro_h(nrestarts), bro_start)
        A_new = [None] * N
        P = G = None
        for n in range(N):
            G = hadamard_gram(A_hat, n)
            P = mttkrp(T, A_hat, n)
            W, _, _ = hals(A[n], P, G, max_inner, tol)
            A_new[n] = W
            A_hat[n] = W + omega * (W - A[n])  # no projection (Sec. 3.3)
        f = f_hat(normT2, P, A_new[N - 1], G)
        restart = f > f_prev
        if restart:
            A_hat = [a.copy() for a in A_new]
            nrestarts += 1
        else:
            A_new = [a.copy() for a in A_hat]
        A = A_new
        f_prev = f
        res.objective.append(f)
        res.restart.append(bool(restart))
        res.weights.append(omega)
        res.hat_min.append(min(float(a.min()) for a in A_hat))
    res.factors = A
    return res
