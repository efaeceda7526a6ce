"""FP64 CPU oracle (test infrastructure only; see invaskit_oracle)."""
from .invaskit_oracle import (  # noqa: F401
    OracleSingular, Factorization, factorize, solve, solve_node, matvec,
    matvec_rows, skeletonize_weights, dense_assemble, gaussian)
