"""Seeded synthetic inputs (geometry, boundary data, forcing) shared by tests and benchmarks."""
from . import geometry, problems  # noqa: F401
from .problems import ProblemSpec  # noqa: F401
