"""FP64 CPU oracle of QFactor-Sample instantiation (arXiv 2405.12866).

TEST INFRASTRUCTURE ONLY. Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It wraps the plain C
implementation in ``qfs_oracle.c`` with ctypes and shares nothing with the HIP
implementation in ``paper_2405_12866_amd``.

Parity is pinned for every function here by the ``-m "not gpu"`` tests (Philox
known-answer vectors, Haar moments, dense brute force, closed forms and invariants);
none is left unpinned.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import build, load  # noqa: F401
