"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only draws random numbers and assembles input tensors; it holds none of the
decomposition method's arithmetic (no MTTKRP, Gram, gradient, CG, ALS or residual code).
"""
from .synth import *  # noqa: F401,F403
