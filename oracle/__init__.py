"""CPU FP64 oracle of the mixed-precision sLdG projection sweep.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never imports it.
"""
from .sldg_oracle import *  # noqa: F401,F403
from .sldg_oracle import TIERS, num_threads  # noqa: F401
