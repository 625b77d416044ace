"""FP64 CPU oracle of the 3D delay-and-sum method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library and never reads
a value produced by it.

See ``oracle.das`` for the definitions and the readings they rest on.
"""
from .das import *  # noqa: F401,F403
