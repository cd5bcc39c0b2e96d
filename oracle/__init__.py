"""CPU FP64 oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the HIP library never does.
"""
from .glam_oracle import *  # noqa: F401,F403
