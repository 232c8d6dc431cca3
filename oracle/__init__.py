"""CPU FP64 oracle for the Krylov-vector path of Gelfgat's cube-convection
stability solver (arXiv:1905.11601).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (``paper_1905_11601_amd``); the only module both sides read is
the seeded input generator ``paper_1905_11601_amd.inputs``, which holds none of
the method's arithmetic.

Everything is plain PyTorch CPU float64 (slicing, arithmetic, matmul) plus
NumPy/SciPy dense linear algebra.  The operators follow the finite-volume
reading of the paper's discretisation written out in the design notes of the
repository (staggered MAC grid with stored wall nodes, central fluxes):

* ``grid``     -- face/centre coordinates, Sec. 4 eq. (22) stretching
* ``ops``      -- residual F of eqs (1)-(3) and its Jacobian, eqs (8)-(9)
* ``tpf``      -- Kronecker Laplacian and its eigenbasis inverse, eqs (14)-(18),
                  and the temperature projection of eqs (19)-(21)
* ``krylov``   -- one Krylov vector, eqs (11)-(13) with the SIMPLE loop of
                  Sec. 3.1, its transpose (reverse-mode AD of the forward
                  definition), Arnoldi/GMRES/BiCGstab(2)/Newton drivers
* ``dense``    -- brute-force dense formulations on tiny grids (pins)

Parity status per function is stated in each module header.
"""
from .grid import Axis, Grid  # noqa: F401
