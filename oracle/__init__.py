"""FP64 CPU oracle for the ASSS two-level solver (Manguoglu & Mehrmann,
"A two-level iterative scheme for general sparse linear systems based on
approximate skew-symmetrizers").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU library computes.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
GPU library never calls it and shares no code with it.

Every function cites the passage of the paper it follows.  Where the paper is
silent or garbled, the reading taken is stated at the function.

Modules
-------
preprocess  validation, max-product matching, canonical scaling (Sec. 2, eq. mc64)
skewsym     least-squares skew-symmetrizer S (Sec. 2 eqs. 1-2, regularized; App. A)
split       A_hat = Abar S, D, Omega, J_tilde, negative-diagonal set (Sec. 3)
lanczos     counter-based start vector and the skew-Lanczos process (Fig. 2)
mrs         simultaneous minimal residual iterations for (alpha I + K) x = b (App. B)
precond     deflated operator, combined low-rank term and its SMW application (Sec. 3.2)
ildl        Bunch-Kaufman incomplete LDL^T of M_hat, |D| factor, low-rank term (Sec. 3, Fig. 1)
solver      outer iterations (flexible GMRES; TFQMR as in the experiments),
            back-transform, adjoint, value gradient of a solve (Sec. 3, Sec. 4.1)
"""
from .preprocess import (StructurallySingular, ZeroDiagonal, validate_csr,
                         max_product_matching, canonical_scaling, permute_scale)
from .skewsym import s_pattern, build_lls, solve_lls, skew_symmetrizer, lls_gradient
from .split import split_ahat
from .lanczos import splitmix64_uniform, start_vector, skew_lanczos
from .mrs import mrs
from .precond import Preconditioner
from .solver import (SolveOptions, SetupOptions, OracleSetup, setup, solve, solve_adjoint,
                     value_gradient, IldlOracleSetup, setup_ildl)
from .ildl import IldlOptions, IldlFactor, ildl, scaled_factor, low_rank

__all__ = [
    "StructurallySingular", "ZeroDiagonal", "validate_csr", "max_product_matching",
    "canonical_scaling", "permute_scale", "s_pattern", "build_lls", "solve_lls",
    "skew_symmetrizer", "lls_gradient", "split_ahat", "splitmix64_uniform",
    "start_vector", "skew_lanczos", "mrs", "Preconditioner", "SolveOptions",
    "SetupOptions", "OracleSetup", "setup", "solve", "solve_adjoint", "value_gradient",
    "IldlOracleSetup", "setup_ildl", "IldlOptions", "IldlFactor", "ildl", "scaled_factor",
    "low_rank",
]
