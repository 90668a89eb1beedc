"""MI355X-native P1 finite-element energies and gradients (arXiv 2109.01158).

The compute path is libp1e.so (HIP kernels for gfx950 behind a C ABI, include/p1e.h); this
package is its thin Python binding. Importing it fails if the library is not built.
"""

from ._lib import (  # noqa: F401
    P1E_FD, P1E_FP64, P1E_FULL_GEOMETRY, P1E_GINZBURG_LANDAU, P1E_INPUT_ORDER, P1E_MIXED,
    P1E_NEOHOOKE, P1E_PLAPLACE, P1E_PLAPLACE_ORTHO, P1E_STATIC_SCRATCH_BYTES, P1E_SVK, P1EError,
    lib,
)
from .api import (  # noqa: F401
    Mesh, Server, energy, energy_forces, grad_exact, grad_exact_static, grad_gather,
    grad_patch_fd, grad_patch_fd4,
    grad_scale, material_constants, mesh_bind, mesh_create, mesh_destroy, mesh_minimize, minimize,
    minimize_workspace_bytes, mesh_get_info, neohooke_constants, prof_collect, prof_enable,
    prof_reset, svk_constants, workspace_bytes,
)
from .autograd import GraphedStep, P1Energy, p1_energy  # noqa: F401

lib()  # fail loudly at import if libp1e.so is missing
