"""FP64 CPU oracle for the particle-by-particle QMC move (arXiv 2209.14487).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The HIP library and its Python
binding never import it.
"""
from .oracle import *  # noqa: F401,F403
