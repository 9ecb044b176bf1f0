"""CPU oracle of the multi-objective Digital Annealer on the bi-objective QAP.

TEST INFRASTRUCTURE ONLY: the plain C reference in ``mda_oracle.c`` and its ctypes
wrapper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.
"""
from .oracle import *  # noqa: F401,F403
