"""FP64 CPU oracle of the 1D radiative PIC step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
from .oracle import Oracle, OracleParams, build_oracle, FLAGS, philox, u24  # noqa: F401
