"""FP64 CPU oracle for the 3D cuboid central-moment LB scheme (D3Q27).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports it and
shares no code, table or helper with it.

The oracle is a plain, slow, explicit-matrix implementation written from the
paper (Yahia, Schupbach, Premnath, "Three-dimensional central moment lattice
Boltzmann method on a cuboid lattice for anisotropic and inhomogeneous flows",
arXiv:2107.14774):

* ``lattice``      -- velocity set (eq. 1), moment bases P, S, Q (eq. 57-61),
                      the combination matrix B of eq. 5 / App. D, and the
                      frame transformation F(u) of the central moments (eq. 3a).
* ``equilibrium``  -- central-moment equilibria (eq. 9), raw equilibria through
                      F(-u), f_eq = Q^-1 m_eq, source moments (eq. 11c).
* ``collision``    -- the collide step of Sec. 3.2 with the App. D collision
                      model (extended equilibria, local strain rates).
* ``streaming``    -- periodic streaming and halfway bounce-back (Sec. 4, U=0).
* ``lbm``          -- initialisation, step, observables (eq. 12), FP64 sums.
* ``direct``       -- an independent route to the same collision through the
                      central-moment definition (eq. 3a) and a dense solve; it
                      exists to pin the factor chain F S P.
* ``gradient``     -- reverse mode through the oracle step (torch autograd).
* ``analytic``     -- closed forms used as pins: eq. 53 parameter map,
                      viscous decay rates, rectangular-duct series.

Every function works in float64 on the CPU with PyTorch tensors (plain torch
ops, no fusion); arrays of populations are laid out ``[27, nz, ny, nx]``.

Parity status: every function is pinned by a ``-m "not gpu"`` test except
where its docstring says "parity unpinned".
"""

from . import lattice, equilibrium, collision, streaming, lbm, direct, analytic  # noqa: F401
from .lbm import Params  # noqa: F401
