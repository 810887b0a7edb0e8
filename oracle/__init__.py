"""FP64 CPU oracle for the HHO elasto-acoustic ERK path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
from .oracle import Oracle, build_oracle, ERK_TABLEAUX  # noqa: F401
