"""Seeded synthetic input generators shared by the oracle tests, the GPU tests and the benchmark.

Holds no arithmetic of the integration method itself; see generate.py.
"""
from .generate import *  # noqa: F401,F403
from .generate import CONFIGS, config_workload, make_workload, rng_for  # noqa: F401
