"""MI355X-native two-site DMRG for the parent Hamiltonian of Gaussian boson
sampling (arXiv 2410.18740), as a thin Python layer over the HIP library
libtn.so.  Torch provides device memory and the stream; all arithmetic of the
method runs in the library's kernels.
"""
from .api import (Context, MPO, MPS, SweepOpts, dmrg_sweep, dmrg_solve, energy, energy_variance, lbo_step, marginals, sample,
                  heff_apply, env_update, truncate, cgemm, philox4x32_10, matvec_flops, env_flops, rdm,
                  squeezed_basis, MLP, ws_features, ws_targets, ws_initial_state, ws_gaussian_params, cutoff_report,
                  noise_uniform_loss, noise_williamson, sample_displaced,
                  PlboOpts, PLBO_ADAM, PLBO_LBFGS, plbo_ops, plbo_minimize, plbo_fock_isometry, plbo_effective_cutoff, plbo_enable, plbo_linear, plbo_linear_isometries, plbo_params, plbo_site_gradient, plbo_sweep,
                  FP64, FP32, BF16X3)
from ._lib import TnError, LIB_PATH

__all__ = ["Context", "MPO", "MPS", "SweepOpts", "dmrg_sweep", "dmrg_solve", "energy", "energy_variance", "lbo_step", "marginals",
           "sample", "heff_apply", "env_update", "truncate", "cgemm", "philox4x32_10", "matvec_flops",
           "env_flops", "rdm", "squeezed_basis", "MLP", "ws_features", "ws_targets", "ws_initial_state", "ws_gaussian_params", "cutoff_report",
           "noise_uniform_loss", "noise_williamson", "sample_displaced",
           "PlboOpts", "PLBO_ADAM", "PLBO_LBFGS", "plbo_ops", "plbo_minimize", "plbo_fock_isometry", "plbo_effective_cutoff", "plbo_enable", "plbo_linear", "plbo_linear_isometries", "plbo_params", "plbo_site_gradient", "plbo_sweep",
           "FP64", "FP32", "BF16X3", "TnError", "LIB_PATH"]
