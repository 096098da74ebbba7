"""FP64 CPU oracle of the two-component pseudopotential LBM step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.
"""
from .oracle import Oracle, OracleParams, lattice_tables  # noqa: F401
