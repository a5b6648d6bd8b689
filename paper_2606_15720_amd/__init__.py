"""MI355X (gfx950) UGKS phase-space step: the C-ABI library and its binding.

``ugks`` is the ctypes binding of ``libugks.so`` (see include/ugks.h); the
HIP sources live in ``csrc/`` and are compiled by ``build.py``.
"""

from . import ugks  # noqa: F401
from .ugks import Solver, UGKSError  # noqa: F401
