"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only draws random numbers and lays them out in arrays.  It holds
none of the transform or multiplication arithmetic, so the oracle and the HIP
path can both take their inputs from here without sharing any of the method.
"""

from .splitmix import SplitMix64, mix64
from . import workloads

__all__ = ["SplitMix64", "mix64", "workloads"]
