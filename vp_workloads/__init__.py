"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark."""
from .generators import *  # noqa: F401,F403
