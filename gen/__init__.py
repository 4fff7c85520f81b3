"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws random numbers and lays out index/value arrays.  It
holds none of the semiring arithmetic of the contraction: duplicate keys are
left in place (the fold combines them), and no product or sum of values is
formed here.
"""

from .synth import *  # noqa: F401,F403
