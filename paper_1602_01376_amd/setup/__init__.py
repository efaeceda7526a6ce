"""Seeded CPU setup: synthetic points, ball tree, ASKIT skeletons and P.

Its output is the input of the factorization; this package holds none of
the INV-ASKIT factor/solve arithmetic.
"""
from .problem import Problem, WORKLOADS, make_problem, rhs_for  # noqa: F401
