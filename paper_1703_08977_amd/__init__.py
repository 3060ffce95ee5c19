"""MI355X-native generalized Feynman-Kac propagation of He walkers.

The C ABI (include/he_fk.h, libhefk.so built for gfx950) does the work; this
package marshals arguments (``api``), holds the seeded workload definitions
(``workloads``) and wraps the pathwise gradient in a torch.autograd.Function
(``autograd``).
"""
from .api import (Ensemble, he_fk_energy, he_fk_energy_blocks, he_fk_grad, he_fk_grad_scratch_bytes, he_fk_init,  # noqa: F401
                  he_fk_propagate, he_fk_propagate_noalloc, he_fk_propagate_workspace_bytes, make_params, run)
from . import workloads  # noqa: F401
