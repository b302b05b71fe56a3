"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .generators import Problem, make, CONFIGS  # noqa: F401
