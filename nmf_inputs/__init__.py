"""Seeded synthetic inputs shared by the CPU oracle's tests and the GPU path.

Only random-number generation and input construction live here (Philox-4x32-10
on host and device, matrix recipes, CSR re-indexing); none of the
factorisation's arithmetic does.
"""
from . import philox, configs  # noqa: F401
from .configs import WORKLOADS, Workload, seed_for  # noqa: F401
