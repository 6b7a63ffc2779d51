"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws positions, charges and weights; it holds none of the
electrostatics or the interpolation arithmetic.
"""
from .systems import System, Site, make_batch, make_config, make_system, CONFIG_NAMES  # noqa: F401
