"""CPU FP64 oracle for the PinT quasi-boundary value methods.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct CPU
reference used to check the GPU library.  Only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it; the
library and its Python binding never do, and it shares no code with them.
"""
from . import qbvm_oracle, mlp_oracle  # noqa: F401
