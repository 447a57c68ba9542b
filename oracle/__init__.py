"""FP64 CPU oracle for the FPW periodogram.

TEST INFRASTRUCTURE: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library
never imports, links or calls it.  Every function is written from the
paper's definitions (Eq. 1, App. A, App. D) and is itself pinned by the
CPU tests against exact arithmetic, independent derivations and closed
forms.
"""
from .fpw_oracle import *  # noqa: F401,F403
from .fpw_oracle import EPS_BIN  # noqa: F401
