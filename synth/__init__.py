"""Seeded synthetic least-squares problems shared by the CPU oracle and the GPU library's tests and
benchmark.  Holds no arithmetic of the method (no sketch, factorisation or solver): it only builds
A, y and, where known exactly, the solution.
"""
from .problems import make_integer_matrix, make_planted, make_problem, singular_values

__all__ = ["make_problem", "make_planted", "make_integer_matrix", "singular_values"]
