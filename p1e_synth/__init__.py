"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This module only *generates* inputs: structured simplex meshes, Dirichlet masks, nodal
loads and seeded nodal fields. It holds none of the method's arithmetic (no element
geometry, no densities, no gradients), so the oracle and the HIP path stay independent
of each other and meet only here.

Every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""

from .meshes import (  # noqa: F401
    rect_tri_mesh,
    kuhn_box_mesh,
    kuhn_bar_level,
    lshape_tri_mesh,
    jitter_interior,
)
from .problems import (  # noqa: F401
    Problem,
    plaplace_square,
    neohooke_beam_2d,
    neohooke_box_3d,
    svk_beam_2d,
    svk_box_3d,
    gl_domain,
    twisted_bar,
    plaplace_lshape,
    config_problem,
    with_load,
    CONFIGS,
)
