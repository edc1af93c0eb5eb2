"""Plain FP64 CPU oracle for the Lindblad optimal-control hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (no kernels, headers, helpers, tables or constants); the two
meet only in the seeded input generators of ``workloads``, which hold none of
the method's arithmetic.

Every function follows the paper (Guenther, Petersson, DuBois, "Quandary: an
open-source C++ package for high-performance optimal control of open quantum
systems") section by section, in its notation, written for readability rather
than speed.  Parity pins: see the module docstring of ``oracle.lindblad``.
"""
from .lindblad import *  # noqa: F401,F403
