"""FP64 CPU oracle for HER-accelerated HALS block-coordinate descent NTF.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct NumPy float64
implementation of what the GPU hot path computes, written from the paper (Ang, Cohen,
Hien, Gillis, "Accelerating block coordinate descent for nonnegative tensor
factorization", arXiv 2001.04321). Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product library never does, and it
shares no code, header, table or helper with the GPU path.

Every function cites the passage it follows (section, equation label or algorithm of
the paper). Inputs are the exact values the GPU sees (float32 / bfloat16 values upcast
to float64); all arithmetic is float64.

Modules
-------
tensor  : Kronecker / Khatri-Rao products, unfoldings, Kruskal reconstruction, the block
          matrix B^(i), MTTKRP, Grams and their Hadamard product, objective, gradient.
hals    : A-HALS column updates and the inner stopping rule.
pgd     : projected gradient and accelerated projected gradient block solvers.
admm    : the ADMM block solver (AO-ADMM / HER-ADMM).
comparators : APG, iBPG and Bro's extrapolation in the block-wise HER structure.
her     : extrapolation, the beta schedule, the restart surrogate F-hat, Algorithm 2 (HER)
          and Algorithm 1 (plain alternating optimization).
metrics : data-fitting error, relative error / fit, factor error with matching.
loss    : the squared-error loss without the 1/2 and its gradient.
tucker  : the Tucker-compressed objective and its gradient (Appendix A).
"""
from .tensor import (kron_columns, khatri_rao, unfold, fold, kruskal, block_matrix, mttkrp,
                     mttkrp_rows, gram, hadamard_gram, objective, gradient)
from .hals import hals_column, hals
from .pgd import lipschitz, pg_step, pgd, nesterov
from .admm import admm, admm_rho
from .tucker import (tucker_full, tucker_her_solve, tucker_mttkrp, tucker_norm2,
                     tucker_relative_error)
from .comparators import apg_solve, ibpg_solve, ibpg_block, bro_solve, bro_omega, bro_h, t_next
from .her import (HERParams, extrapolate, update_beta, f_hat, her_solve, ao_solve,
                  HERResult)
from .metrics import residual_norm, relative_error, fit, factor_error
from .loss import cp_loss, cp_loss_grad

__all__ = [
    "kron_columns", "khatri_rao", "unfold", "fold", "kruskal", "block_matrix", "mttkrp",
    "mttkrp_rows",
    "gram", "hadamard_gram", "objective", "gradient", "hals_column", "hals", "HERParams",
    "extrapolate", "update_beta", "f_hat", "her_solve", "ao_solve", "HERResult",
    "residual_norm", "relative_error", "fit", "factor_error", "cp_loss", "cp_loss_grad",
    "lipschitz", "pg_step", "pgd", "nesterov", "admm", "admm_rho", "apg_solve", "ibpg_solve",
    "ibpg_block", "bro_solve", "bro_omega", "bro_h", "t_next", "tucker_full", "tucker_mttkrp",
    "tucker_norm2", "tucker_her_solve", "tucker_relative_error",
]
