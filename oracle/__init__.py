"""CPU oracle for the staggered periodic incompressible Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
its Python binding) may import, call or link this package; only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.

Plain, slow, float64 numpy (and torch-CPU float64 for the CNN closure): each
function states the passage of the paper it follows. It shares no code with
the HIP path.
"""
from .ins import (  # noqa: F401
    spacing_of,
    divergence,
    gradient,
    diffusion,
    convection,
    rhs,
    laplace_eigenvalues,
    poisson_solve,
    project,
    step_rk4,
    divergence_vjp,
    gradient_vjp,
    diffusion_vjp,
    convection_vjp,
    rhs_vjp,
    poisson_solve_vjp,
    project_vjp,
    step_rk4_vjp,
    rk4_stages,
    wray3_stages,
    step_wray3,
    step_wray3_vjp,
    WRAY3_G,
    WRAY3_Z,
    kinetic_energy,
    rollout_loss,
    rollout_loss_grad,
)
from .aux import face_filter, energy_spectrum  # noqa: F401
from . import eddy  # noqa: F401,E402
from . import walls  # noqa: F401,E402
