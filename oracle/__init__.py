"""Independent FP64 CPU oracle of the microwave-tomography solve path.

TEST INFRASTRUCTURE ONLY: it exists to check the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or run anything under ``oracle/``; the GPU
product path never does, and the two share no code (only the seeded input
generators of ``mw_inputs`` feed both).

Modules:
  fem      -- edge-element assembly, sources, port projections (Section 2, 4)
  dd       -- overlapping decomposition, partition of unity, ORAS (Section 3)
  gmres    -- right-preconditioned pseudo-block GMRES(m) with CGS2 (Section 6)
              and block GMRES(m) (the block Krylov method of Section 7)
  inverse  -- S-matrix, misfit, adjoint gradient, Woodbury finite differences
              (Sections 4-5)
"""
from . import dd, fem, gmres, inverse  # noqa: F401
