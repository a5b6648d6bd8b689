"""CPU FP64 oracle of the UGKS phase-space step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product path (``paper_2606_15720_amd``) never imports it.
"""

from .oracle import Oracle, build_oracle, lib_path, gamma, half_moments, interface_state, \
    slopes, gram, gram_u, threads, set_threads  # noqa: F401
from . import learned  # noqa: F401,E402
