"""MI355X (gfx950) ISDF-SMW inverse of the dielectric matrix.

The compute path is the HIP library libisdfsmw.so (C ABI: include/isdf_smw.h);
this package only marshals arguments to it (see binding.py).
"""
from .binding import (IsdfError, MultiGraph, Plan, Problem, Report, Result, check_inputs, contour_nodes, core_m, coulomb_u,  # noqa: F401
                      eps_inv, eps_inv_grad, eps_inv_loss, eps_inv_multi, eps_inv_noalloc, fit_theta, grad_workspace_bytes,
                      gvectors, header_functions, lib, make_problem, problem_for, sigma_cohsex, sigma_workspace_bytes,
                      smw_apply, workspace_bytes)
