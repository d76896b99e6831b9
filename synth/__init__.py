"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the method: only parameter draws,
initial lattices and manifests of the workloads (numpy ``default_rng``).
"""
from .workloads import *  # noqa: F401,F403
