"""CPU oracle for bulk direct-method simulation of CWC models.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are its only users.  The GPU library neither
imports nor links anything from here.
"""
from .cwc import (FlatModel, build, draw, finalize, philox, select, simulate,  # noqa: F401
                  ssa_log, STATUS)
from .gcwc import GModel, gsimulate  # noqa: F401
