"""Plain FP64 CPU oracle for prolate-spheroidal Slater integrals.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the benchmark may
load it.  The product path never imports it and never falls back to it.
"""
from .binding import *  # noqa: F401,F403
from .ri import pair_index, pairs_matrix, forward_substitution, ri_assemble  # noqa: F401,E402
