"""Heuristic extrapolation with restarts (HER, Algorithm 2) around A-HALS, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of points the paper leaves open (each one a single place in this file):
* F-hat_0 is not defined by Algorithm 2's initialization; it is taken as F(A_0).
* The restart test is strict: F-hat_k > F-hat_{k-1} restarts, equality accepts
  (Algorithm 2 and eqs. HER_eq:beta_update / HER_eq:beta_bar_update agree on this).
* After a restart the stored F-hat_{k} is still the value computed at iteration k.
* beta is one scalar per problem (Algorithm 2 carries a single beta_k).
* Parameter ordering follows Sec. 3.1.4 and eq. HER:relation (1 <= gamma_bar <= gamma
  <= eta); Algorithm 2's initialization line prints the first two the other way round.
* A^(i)_0-hat = A^(i)_0 (Sec. 3.1.4, last remark), beta_bar_0 = 1 (Algorithm 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .admm import admm
from .hals import hals
from .pgd import nesterov, pgd
from .tensor import hadamard_gram, mttkrp, objective, gram


@dataclass(frozen=True)
class HERParams:
    """HER parameters with the paper's defaults (Sec. 3.1.4 and Sec. 4.1) and the inner
    stopping rule of Sec. 4.1 (50 sweeps, relative tolerance 1e-2)."""
    beta0: float = 0.5
    gamma: float = 1.05
    gamma_bar: float = 1.01
    eta: float = 1.5
    max_inner: int = 50
    inner_tol: float = 1e-2
    # block solver: "ahals" (Sec. 2.1.4), "pgd" or "nesterov" (projected gradient steps,
    # Sec. 2.2; HER-PGD50 / HER-Nesterov50 of Sec. 3.1.4), "admm" (ADMM steps, Sec. 2.1.2;
    # HER-ADMM)
    inner: str = "ahals"

    def validate(self) -> None:
        if self.inner not in SOLVERS:
            raise ValueError(f"inner must be one of {sorted(SOLVERS)}")
        if not (0.0 <= self.beta0 < 1.0):
            raise ValueError("beta0 must lie in [0, 1)")
        if not (1.0 <= self.gamma_bar <= self.gamma <= self.eta):
            raise ValueError("need 1 <= gamma_bar <= gamma <= eta")
        if self.max_inner < 1 or self.inner_tol < 0.0:
            raise ValueError("max_inner >= 1 and inner_tol >= 0 required")


SOLVERS = {"ahals": hals, "pgd": pgd, "nesterov": nesterov, "admm": admm}


def extrapolate(A_new: np.ndarray, A_old: np.ndarray, beta: float) -> np.ndarray:
    """Extrapolate-project step, eq. extproj_her: max(0, A_k + beta_{k-1} (A_k - A_{k-1}))."""
    A_new = np.asarray(A_new, dtype=np.float64)
    A_old = np.asarray(A_old, dtype=np.float64)
    return np.maximum(0.0, A_new + beta * (A_new - A_old))


def update_beta(beta: float, beta_bar: float, restart: bool, p: HERParams):
    """One step of the beta / beta_bar schedule (eqs. HER_eq:beta_update and
    HER_eq:beta_bar_update, Algorithm 2 restart branch).

    restart: beta_bar <- beta, beta <- beta / eta.
    accept : beta <- min(beta_bar_old, gamma * beta), beta_bar <- min(1, gamma_bar * beta_bar_old).
    """
    if restart:
        return beta / p.eta, beta
    return min(beta_bar, p.gamma * beta), min(1.0, p.gamma_bar * beta_bar)


def f_hat(normT2: float, P_last: np.ndarray, A_last: np.ndarray, G_last: np.ndarray) -> float:
    """Restart surrogate from quantities of the last block's update (Sec. 3.1.3).

    With P = T_[N] B^(N) and G = (B^(N))^T B^(N) built from the other blocks' current
    values, expanding 1/2 ||T_[N] - A B^T||^2 gives
    F = 1/2 (||T||^2 - 2 <P, A> + <G, A^T A>).
    """
    P_last = np.asarray(P_last, dtype=np.float64)
    A_last = np.asarray(A_last, dtype=np.float64)
    G_last = np.asarray(G_last, dtype=np.float64)
    return 0.5 * (float(normT2) - 2.0 * float(np.sum(P_last * A_last))
                  + float(np.sum(G_last * gram(A_last))))


@dataclass
class HERResult:
    factors: list
    fhat: list = field(default_factory=list)        # F-hat_k, k = 1..K
    restart: list = field(default_factory=list)     # True if iteration k restarted
    beta: list = field(default_factory=list)        # beta_k after iteration k's update
    beta_bar: list = field(default_factory=list)    # beta_bar_k after iteration k's update
    sweeps: list = field(default_factory=list)      # per iteration: inner sweeps per block
    fhat0: float = 0.0
    state: dict = field(default_factory=dict)       # resumable state after the last iteration


def her_solve(T: np.ndarray, A0, iters: int, params: HERParams = HERParams(),
              state: dict | None = None, hook=None, mttkrp_fn=None,
              normT2: float | None = None) -> HERResult:
    """Algorithm 2 (HER) with A-HALS (or, by `params.inner`, projected gradient or ADMM
    steps) as the block solver, for `iters` outer iterations.

    Iteration k, block n = 1..N (eq. NNLS_her_exact): the block problem uses the
    extrapolated blocks of this iteration for l < n and of the previous iteration for
    l > n; A-HALS warm-starts from A_{k-1}^(n) (Algorithm 1's note, Sec. 2.1.4); then
    eq. extproj_her extrapolates with beta_{k-1}. After the last block, F-hat_k =
    F(A-hat_k^(1..N-1), A_k^(N)) (Algorithm 2) is formed from the last block's P and G
    (Sec. 3.1.3), compared with F-hat_{k-1}, and the iterates and beta are updated.

    `state` (from a previous result's .state) resumes a run: factors, beta, beta_bar,
    F-hat_{k-1}. Without it the run starts from A0 with beta0, beta_bar = 1,
    F-hat_0 = F(A_0).

    `hook(k, A_prev, A_new, A_hat, fhat_k)` (optional) sees each iteration's blocks just
    before the restart decision: A_{k-1}, A_k, A-hat_k and F-hat_k.

    `mttkrp_fn(A, n)` and `normT2` replace the dense tensor's MTTKRP and ||T||^2 when the
    data is given in another format (T then only supplies its order via len(A0));
    F-hat_0 = F(A_0) is then formed by the same Gram-trick expansion as F-hat_k.
    """
    params.validate()
    if mttkrp_fn is None:
        T = np.asarray(T, dtype=np.float64)
        N = T.ndim
        normT2 = float(np.sum(T * T))
        mttkrp_fn = lambda A_, n_: mttkrp(T, A_, n_)  # noqa: E731
        dense = True
    else:
        N = len(A0) if state is None else len(state["factors"])
        dense = False
    if state is None:
        A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
        beta, beta_bar = params.beta0, 1.0
        if dense:
            fhat_prev = objective(T, A)
        else:
            fhat_prev = f_hat(normT2, mttkrp_fn(A, N - 1), A[N - 1], hadamard_gram(A, N - 1))
    else:
        A = [np.array(a, dtype=np.float64, copy=True) for a in state["factors"]]
        beta, beta_bar, fhat_prev = state["beta"], state["beta_bar"], state["fhat"]
    A_hat = [a.copy() for a in A]
    res = HERResult(factors=[], fhat0=fhat_prev)
    for _k in range(iters):
        A_new = [None] * N
        sweeps_k = []
        P_last = G_last = None
        for n in range(N):
            # A_hat holds A-hat_k^(l) for l < n and A-hat_{k-1}^(l) for l > n.
            G = hadamard_gram(A_hat, n)
            P = mttkrp_fn(A_hat, n)
            solver = SOLVERS[params.inner]
            W, s, _ = solver(A[n], P, G, params.max_inner, params.inner_tol)
            sweeps_k.append(s)
            A_new[n] = W
            A_hat[n] = extrapolate(W, A[n], beta)
            if n == N - 1:
                P_last, G_last = P, G
        fh = f_hat(normT2, P_last, A_new[N - 1], G_last)
        if hook is not None:
            hook(_k + 1, A, A_new, A_hat, fh)
        restart = fh > fhat_prev
        if restart:
            A_hat = [a.copy() for a in A_new]
        else:
            A_new = [a.copy() for a in A_hat]
        beta, beta_bar = update_beta(beta, beta_bar, restart, params)
        A = A_new
        fhat_prev = fh
        res.fhat.append(fh)
        res.restart.append(bool(restart))
        res.beta.append(beta)
        res.beta_bar.append(beta_bar)
        res.sweeps.append(sweeps_k)
    res.factors = A
    res.state = dict(factors=[a.copy() for a in A], beta=beta, beta_bar=beta_bar,
                     fhat=fhat_prev)
    return res


def ao_solve(T: np.ndarray, A0, iters: int, max_inner: int = 50, inner_tol: float = 1e-2,
             record_objective: bool = False):
    """Algorithm 1 (alternating optimization) with A-HALS blocks: block n is solved with the
    latest values of every other block (eq. NNLS), warm-started from its previous value.

    Returns (factors, objective values after each iteration if requested, sweeps).
    """
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
    objs, sweeps = [], []
    for _k in range(iters):
        s_k = []
        for n in range(N):
            G = hadamard_gram(A, n)
            P = mttkrp(T, A, n)
            A[n], s, _ = hals(A[n], P, G, max_inner, inner_tol)
            s_k.append(s)
        sweeps.append(s_k)
        if record_objective:
            objs.append(objective(T, A))
    return A, objs, sweeps
