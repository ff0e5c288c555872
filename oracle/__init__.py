"""FP64 CPU oracle of the RBF terrain hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg. The GPU library never imports, links or
executes anything in this package, and this package imports nothing from it.
"""
from .rbf_oracle import *  # noqa: F401,F403
