"""MI355X-native fused collide-and-stream step of the 3D cuboid central-moment
lattice Boltzmann scheme on a D3Q27 lattice (arXiv:2107.14774).

The compute path is the HIP library ``liblbm.so`` (C ABI in include/lbm.h,
sources in ``csrc/``); ``lbm`` is its Python binding and ``adjoint`` the
autograd wrapper with checkpointing.
"""

from .lbm import (Lattice, Handle, relaxation_rates, lbm_relaxation_rates, lbm_create, lbm_init,  # noqa: F401
                  lbm_import, lbm_export, lbm_export_nodes, lbm_step, lbm_set_force, lbm_step_forcing, lbm_density, lbm_step_full,
                  lbm_stream, lbm_copy, lbm_moments, lbm_check_sums, lbm_step_adjoint, lbm_step_adjoint_full,
                  lbm_step_adjoint_full_noalloc, lbm_density_adjoint, lbm_adjoint_stream, lbm_moments_adjoint,
                  lbm_init_adjoint, lbm_adjoint_to_natural, lbm_adjoint_from_natural, lbm_set_step_counter,
                  lbm_step_counter)
