"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the ghost-cell method: only grids, body
parameters, analytic fields, boundary data evaluated from analytic fields at
given points, and surface quadrature rules.
"""
from .workloads import *  # noqa: F401,F403
