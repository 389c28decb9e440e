"""FP64 CPU oracle for the fermion-determinant-ratio path of Leder, Finkenrath
and Knechtli, "Fermions as global correction in lattice QCD" (Lattice 2011).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library: the stencil, solvers and Philox live in plain C
(``wdr_oracle.c``), the orchestration in plain numpy (``core.py``).

Parity status of each function is listed in ``core.py``'s module docstring.
"""
from .core import *  # noqa: F401,F403
