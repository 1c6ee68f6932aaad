"""Seeded synthetic inputs for nonnegative CP factorization (NTF) experiments.

This module only *draws data*: planted nonnegative factors, the dense tensor they span,
Gaussian noise at a target signal-to-noise ratio, and random initial factors. It follows
the synthetic-data recipe of the paper's experimental set-up (Sec. 4.1, "Generate a
synthetic data": planted factors i.i.d. U[0,1], T = max(0, T_clean + sigma*E) with E
standard normal; "Initialization": initial factors i.i.d. U[0,1]).

It holds no step of the factorization method itself (no MTTKRP, Gram, HALS, HER or error
evaluation). Both the FP64 CPU oracle's tests and the GPU path's tests and benchmark take
their inputs from here, so the two sides see the same bytes.

Reading of the paper used here (the paper states absolute noise levels, the workloads
state SNRs in dB): sigma = ||T_clean||_F / (||E||_F * 10**(snr_db/20)), which makes the
realised SNR exact, then the result is clipped at 0 for every workload (Sec. 4.1).

Seeding: numpy.random.Generator(PCG64(seed)). A data seed draws the planted factors in
mode order (row-major per factor), then the optional zero mask, then the noise tensor.
An init seed draws the initial factors in mode order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "generator", "uniform_factors", "correlated_factors", "apply_zero_mask",
    "planted_tensor", "add_noise", "make_problem", "bf16_bits", "bf16_to_f32",
    "round_to_bf16", "WORKLOADS", "workload", "batch_specs", "batch_problem",
    "TuckerProblem", "make_tucker_problem", "TUCKER_WORKLOADS", "tucker_workload",
]


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_factors(g: np.random.Generator, dims, r: int) -> list[np.ndarray]:
    """Factors with i.i.d. U[0,1) entries, one I_n x r float64 matrix per mode."""
    return [g.random((int(I), int(r))) for I in dims]


def correlated_factors(g: np.random.Generator, dims, r: int, rho: float = 0.9) -> list[np.ndarray]:
    """Nonnegative factors whose columns are pairwise correlated with coefficient rho.

    A = sqrt(rho) * c 1^T + sqrt(1 - rho) * U with c (I x 1) and U (I x r) i.i.d. U[0,1):
    every column has variance Var(U[0,1]) and every pair of columns has covariance
    rho * Var(U[0,1]), so the population Pearson correlation is exactly rho, and all
    entries stay nonnegative. Per mode, c is drawn before U.
    """
    out = []
    for I in dims:
        c = g.random((int(I), 1))
        U = g.random((int(I), int(r)))
        out.append(np.sqrt(rho) * c + np.sqrt(1.0 - rho) * U)
    return out


def apply_zero_mask(g: np.random.Generator, factors, frac: float) -> int:
    """Zero each factor entry independently with probability `frac` (in place).

    Returns the number of zeroed entries.
    """
    n = 0
    for A in factors:
        m = g.random(A.shape) < frac
        A[m] = 0.0
        n += int(m.sum())
    return n


def planted_tensor(factors) -> np.ndarray:
    """Dense C-order tensor sum_p a_p^(1) o ... o a_p^(N) in float64 (last mode fastest)."""
    dims = tuple(A.shape[0] for A in factors)
    r = factors[0].shape[1]
    # rows of `rest` enumerate (j_2, ..., j_N) with j_N fastest, matching C order
    rest = factors[-1]
    for A in reversed(factors[1:-1]):
        rest = (A[:, None, :] * rest[None, :, :]).reshape(-1, r)
    return (factors[0] @ rest.T).reshape(dims)


def add_noise(g: np.random.Generator, T_clean: np.ndarray, snr_db, clip: bool = True):
    """T = max(0, T_clean + sigma E), E ~ N(0,1), sigma set so the SNR is exactly snr_db.

    Returns (T, sigma, n_clipped). snr_db=None means noiseless (sigma = 0).
    """
    if snr_db is None:
        T = T_clean.copy()
        sigma = 0.0
    else:
        E = g.standard_normal(T_clean.shape)
        sigma = float(np.linalg.norm(T_clean.ravel()) /
                      (np.linalg.norm(E.ravel()) * 10.0 ** (snr_db / 20.0)))
        T = T_clean + sigma * E
        del E
    n_clipped = 0
    if clip:
        neg = T < 0
        n_clipped = int(neg.sum())
        T[neg] = 0.0
    return T, sigma, n_clipped


@dataclass
class Problem:
    """One synthetic NTF instance. `T` is float64; `A_true` / `A0` are float64 factors."""
    T: np.ndarray
    A_true: list
    A0: list
    r: int
    sigma: float
    n_clipped: int
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        return self.T.shape


def make_problem(dims, r: int, snr_db=None, kind: str = "uniform", mask_frac: float = 0.0,
                 rho: float = 0.9, data_seed: int = 0, init_seed: int = 1,
                 clip: bool = True) -> Problem:
    """Draw planted factors, the noisy tensor and an initial point.

    kind: "uniform" (i.i.d. U[0,1)) or "correlated" (pairwise column correlation rho).
    mask_frac: probability of zeroing each planted-factor entry (drawn after the values).
    """
    dims = tuple(int(d) for d in dims)
    g = generator(data_seed)
    if kind == "uniform":
        A_true = uniform_factors(g, dims, r)
    elif kind == "correlated":
        A_true = correlated_factors(g, dims, r, rho)
    else:
        raise ValueError(f"unknown factor kind {kind!r}")
    n_masked = apply_zero_mask(g, A_true, mask_frac) if mask_frac > 0 else 0
    T_clean = planted_tensor(A_true)
    T, sigma, n_clipped = add_noise(g, T_clean, snr_db, clip=clip)
    del T_clean
    A0 = uniform_factors(generator(init_seed), dims, r)
    meta = dict(dims=dims, r=r, snr_db=snr_db, kind=kind, mask_frac=mask_frac,
                n_masked=n_masked, data_seed=data_seed, init_seed=init_seed)
    return Problem(T=T, A_true=A_true, A0=A0, r=r, sigma=sigma, n_clipped=n_clipped, meta=meta)


# ---------------------------------------------------------------------------------------
# bfloat16 storage (round-to-nearest-even of the float32 value, as the stored tensor type)
# ---------------------------------------------------------------------------------------

def bf16_bits(x) -> np.ndarray:
    """float32 -> uint16 bfloat16 bit patterns, round to nearest, ties to even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    out = ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return out.reshape(x.shape)


def bf16_to_f32(bits) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32).reshape(bits.shape)


def round_to_bf16(x) -> np.ndarray:
    """float32 array of the values a bfloat16 copy of float32(x) holds."""
    return bf16_to_f32(bf16_bits(np.asarray(x, dtype=np.float32)))


# ---------------------------------------------------------------------------------------
# Named workloads (shapes, ranks and noise of the benchmark configurations)
# ---------------------------------------------------------------------------------------

WORKLOADS = {
    # 3-way 50^3, r=10, uniform factors, 40 dB; the small case the oracle runs in seconds
    "cube50_r10": dict(dims=(50, 50, 50), r=10, snr_db=40.0, kind="uniform", iters=200),
    # 3-way 400^3, r=32, pairwise column correlation 0.9, 30 dB; float32 and bf16 forms
    "cube400_r32_corr": dict(dims=(400, 400, 400), r=32, snr_db=30.0, kind="correlated",
                             iters=500),
    # 4-way 128^4, r=64, 30% zeroed factor entries, 20 dB, clipped; stored in bf16
    "quad128_r64_sparse": dict(dims=(128, 128, 128, 128), r=64, snr_db=20.0,
                               kind="uniform", mask_frac=0.3, iters=200),
    # 3-way 512^3, r=50, 30 dB: loss/gradient workload
    "cube512_r50": dict(dims=(512, 512, 512), r=50, snr_db=30.0, kind="uniform", iters=1),
    # 24^3, r=4: finite-difference gradient instance
    "cube24_r4": dict(dims=(24, 24, 24), r=4, snr_db=30.0, kind="uniform", iters=1),
}


def workload(name: str, data_seed: int = 0, init_seed: int = 1) -> Problem:
    w = dict(WORKLOADS[name])
    w.pop("iters")
    return make_problem(data_seed=data_seed, init_seed=init_seed, **w)


def batch_specs(n: int = 256, meta_seed: int = 0, lo: int = 32, hi: int = 160,
                rlo: int = 5, rhi: int = 20) -> list[tuple]:
    """(I1, I2, I3, r) for a batch of independent 3-way problems, drawn uniformly."""
    g = generator(meta_seed)
    out = []
    for _ in range(n):
        dims = g.integers(lo, hi + 1, size=3)
        r = int(g.integers(rlo, rhi + 1))
        out.append((int(dims[0]), int(dims[1]), int(dims[2]), r))
    return out


def batch_problem(spec, b: int, snr_db: float = 30.0) -> Problem:
    """Problem b of a batch: data seed 1000+b, init seed 2000+b."""
    I1, I2, I3, r = spec
    return make_problem((I1, I2, I3), r, snr_db=snr_db, kind="uniform",
                        data_seed=1000 + b, init_seed=2000 + b)


# ---------------------------------------------------------------------------------------
# Data given in Tucker format (the compressed input of the paper's Appendix A)
# ---------------------------------------------------------------------------------------

@dataclass
class TuckerProblem:
    """T = (U^(1) (x) ... (x) U^(N)) core; float64 core (r_1 x ... x r_N) and bases
    (n_p x r_p, orthonormal columns), the planted factors and an initial point."""
    core: np.ndarray
    bases: list
    A_true: list
    A0: list
    r: int
    sigma: float
    meta: dict = field(default_factory=dict)


def make_tucker_problem(dims, ranks, r: int, snr_db=None, data_seed: int = 0,
                        init_seed: int = 1) -> TuckerProblem:
    """A planted nonnegative CP tensor given in Tucker format, with noise in the core.

    Data seed: planted factors A_p ~ U[0,1] (n_p x r) in mode order, then per mode a
    Gaussian n_p x (r_p - r) block; U_p is the orthonormal basis (QR) of [A_p, block], so
    span(U_p) contains the columns of A_p and (U_p U_p^T) A_p = A_p. The core is the planted
    CP of the projected factors U_p^T A_p plus Gaussian noise E at `snr_db` relative to the
    clean core (orthonormal bases keep the SNR of the full tensor); no clipping (the
    format need not be nonnegative). Init seed: A_0 ~ U[0,1] in mode order.
    """
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(x) for x in ranks)
    if any(rp < r for rp in ranks):
        raise ValueError("Tucker ranks must be at least the CP rank")
    g = generator(data_seed)
    A_true = uniform_factors(g, dims, r)
    bases = []
    for A, rp in zip(A_true, ranks):
        X = np.concatenate([A, g.standard_normal((A.shape[0], rp - r))], axis=1)
        Q, _ = np.linalg.qr(X)
        bases.append(Q)
    core_clean = planted_tensor([U.T @ A for U, A in zip(bases, A_true)])
    sigma = 0.0
    if snr_db is None:
        core = core_clean
    else:
        E = g.standard_normal(core_clean.shape)
        sigma = float(np.linalg.norm(core_clean.ravel()) /
                      (np.linalg.norm(E.ravel()) * 10.0 ** (snr_db / 20.0)))
        core = core_clean + sigma * E
    A0 = uniform_factors(generator(init_seed), dims, r)
    meta = dict(dims=dims, ranks=ranks, r=r, snr_db=snr_db, data_seed=data_seed,
                init_seed=init_seed)
    return TuckerProblem(core=core, bases=bases, A_true=A_true, A0=A0, r=r, sigma=sigma,
                         meta=meta)


TUCKER_WORKLOADS = {
    # the shape of the paper's compressed video tensor (Sec. 4.2, "On big data"): 153 x 238
    # x 14000, CP rank 10, Tucker ranks 30, 30 dB
    "tucker_video_r10": dict(dims=(153, 238, 14000), ranks=(30, 30, 30), r=10, snr_db=30.0,
                             iters=200),
}


def tucker_workload(name: str, data_seed: int = 0, init_seed: int = 1) -> TuckerProblem:
    w = dict(TUCKER_WORKLOADS[name])
    w.pop("iters")
    return make_tucker_problem(data_seed=data_seed, init_seed=init_seed, **w)
