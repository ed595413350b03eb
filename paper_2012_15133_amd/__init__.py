"""MI355X-native time stepper for the square phase field crystal equation with the
SAV-BDF2 scheme of Wang, Huang and Wang (arXiv 2012.15133).

The GPU path is the HIP library libspfc.so (C ABI in include/spfc.h); `binding`
wraps it.  `inputs` draws the seeded synthetic initial data.
"""

from .binding import (  # noqa: F401
    Batch, Solver, SpfcError, load_library, make_grid, make_params,
    spfc_workspace_bytes, spfc_init, spfc_step, spfc_mass, spfc_energy, spfc_history,
    spfc_step_count, spfc_get_phi, spfc_state_bytes, spfc_save_state, spfc_load_state,
    spfc_status, spfc_profile, spfc_kernel_times, spfc_strerror, spfc_destroy, spfc_set_graph,
    spfc_batch_workspace_bytes, spfc_batch_init, spfc_batch_step, spfc_batch_set_graph,
    spfc_batch_step_count, spfc_batch_status, spfc_batch_mass, spfc_batch_energy, spfc_batch_history,
    spfc_batch_get_phi, spfc_batch_destroy, spfc_batch_profile, spfc_batch_kernel_times,
    spfc_tune_bytes, spfc_tune, spfc_get_plan, spfc_batch_tune_bytes, spfc_batch_tune, spfc_batch_get_plan,
    spfc_time_kernels, spfc_batch_time_kernels, spfc_batch_reset, spfc_batch_energies, spfc_batch_get_phi_all, spfc_forcing_bytes, spfc_set_forcing,
    spfc_step_forced,
)
