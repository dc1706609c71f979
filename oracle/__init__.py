"""FP64 CPU oracle for BLF-LS (arXiv 1812.07122).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It shares no code with the
GPU path.  Every function follows the passage it cites and is pinned by
``tests/test_oracle.py`` against closed forms, brute force and invariants; no
function here is left unpinned.
"""
from .blfls_oracle import *  # noqa: F401,F403
from .blfls_oracle import __all__  # noqa: F401
