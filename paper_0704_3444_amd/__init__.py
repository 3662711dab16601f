"""MI355X (gfx950) implementation of the symmetric free-energy
multicomponent lattice Boltzmann method (Li & Wagner, arXiv:0704.3444).

The step runs in hand-written HIP kernels (liblbm.so, C ABI in
include/lb.h); this package is the Python binding."""
from .lb import (  # noqa: F401
    Batch, LBError, Lines, Simulation, lb_batch_config_count, lb_batch_config_info, lb_free, lb_get_f, lb_get_state,
    lb_init, lb_lattice_tables, lb_moments, lb_path_in_use, lb_set_state, lb_state_bytes, lb_step,
    lb_workspace_bytes, load, make_params,
)
