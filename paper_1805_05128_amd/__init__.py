"""MI355X (gfx950) contact-SPH hot path: binning, neighbour search, pair
rates, step, Voronoi ownership and their adjoints, behind the C ABI of
include/csph.h (libcsph.so, hand-written HIP)."""
from ._native import (CSPH_OK, CSPH_EINVAL, CSPH_ECAPACITY, CSPH_EDEVICE,  # noqa: F401
                      CSPH_ENONPHYS, CsphError, NonPhysicalState)
from .api import (EOS_IDEAL, EOS_STIFFENED, EOS_MIE_GRUNEISEN, Params, State, StepScalars, Workspace,  # noqa: F401
                  csph_bin, csph_grid_build, csph_init_energy, csph_neighbors, csph_rates,
                  csph_step, default_workspace, profile_enable, profile_groups, profile_read, state_from_workload, version, voronoi_assign,
                  workspace_size, csph_rates_vjp, csph_step_vjp, csph_step_vjp_cfl,
                  csph_init_energy_vjp,
                  zeros_grad, GRAD_FIELDS, BalanceParams, csph_balance_stats,
                  csph_balance_move, adjacency_matrix, csph_vlist_build, csph_step_vlist,
                  VerletRun, csph_step_static, csph_step_voronoi, vlist_ctl,
                  vlist_ctl_read, csph_step_mesh, domain_mesh)
from .autograd import CSPHRollout, rollout  # noqa: F401
