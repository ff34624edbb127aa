"""CPU oracle for the SWCS hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
under ``paper_2411_07920_amd/``; the only inputs both sides share are the
seeded arrays of ``paper_2411_07920_amd.inputs``, passed in as plain arrays.

Parity status of each oracle function is listed in ``oracle/core.py``.
"""
from .core import *  # noqa: F401,F403
from .core import build, load  # noqa: F401
