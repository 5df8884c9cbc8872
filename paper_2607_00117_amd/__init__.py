"""MI355X (gfx950) Schwarzschild orbit-superposition model builder.

A thin ctypes binding over libschw.so.  Every step of the hot path runs in the
library's HIP kernels; this module only marshals arguments.  PyTorch supplies
device memory and the current stream.  If the library is not built, importing
the binding raises: there is no fallback path.
"""
from ._lib import (  # noqa: F401
    SW_F32, SW_F64, SW_GRAM_BF16, SW_GRAM_BF16X3, SW_GRAM_F32, SW_SOLVE_DENSE, SW_SOLVE_NO_ACCEL, SW_FLAG_DRIFT, SW_FLAG_NONFINITE, SW_GRID_CARTESIAN, SW_GRID_CYLINDRICAL,
    SchwError, build_potential, integrate_and_bin, integrate_workspace_bytes, solve_weights,
    solve_workspace_bytes, solve_weights_batched, solve_batched_workspace_bytes, chi2, chi2_workspace_bytes, chi2_noalloc, chi2_noalloc_max_con, model_observables, bin_points, cell_masses, jeans_ics, dither_ics, bundle_rows, integrate_bs23_and_bin, integrate_bs23_workspace_bytes, integrate_orbits,
    obs_spec, ncon, count_quantum, library_path, load, mlp_param_count, mlp_workspace_bytes, mlp_forward, mlp_backward,
    mlp_adam_step, mlp_pack_bf16, mlp_infer_bf16, mlp_mse_grad, set_tuning, get_tuning, gh_moments,
    gh_workspace_bytes, gh_fit_matrix, gh_fit_workspace_bytes, solve_weights_multi, solve_multi_workspace_bytes, bootstrap_data, chi2_model,
)
