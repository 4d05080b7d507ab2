"""Seeded synthetic workloads shared by the simulator tests, the FP64 checker
and the benchmark.  Holds no simulation arithmetic."""
from .circuits import *  # noqa: F401,F403
