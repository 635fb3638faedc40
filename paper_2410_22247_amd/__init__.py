"""MI355X (gfx950) MaxCut-QAOA statevector estimator with orbit-reduced observables.

The compute path is the HIP C-ABI library ``libaaqaoa.so`` (declared in
``include/aaqaoa.h``); this package only marshals arguments to it.  PyTorch
provides device memory and streams.  Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from .api import (  # noqa: F401
    AAQ_AGG_FUSED, AAQ_AGG_PASS_PER_TERM, AAQ_AGG_PER_TERM, AAQ_OBS_HC, AAQ_OBS_HRED, AAQ_PREC_C64, AAQ_PREC_C128,
    AAQError, Problem, aaq_cut_values, aaq_cut_values_layout, aaq_energy, aaq_energy_grad, aaq_num_sets,
    aaq_plan_create, aaq_plan_destroy, aaq_plan_execute, aaq_plan_workspace_size, aaq_state_bytes, aaq_validate,
    aaq_version, aaq_workspace_size, aaq_timing_enable, aaq_timing_read, aaq_timing_classes, aaq_set_tile_bits,
    aaq_get_tile_bits, aaq_autotune, aaq_plan_autotune, aaq_checkpoint_bytes, aaq_energy_grad_checkpointed, Estimator,
    Plan, aaq_lightcone_info, aaq_lightcone_workspace_size, aaq_lightcone_create, aaq_lightcone_execute,
    aaq_lightcone_destroy, LightCone, aaq_edge_orbits, aaq_rcc_eta, aaq_sample_workspace_size, aaq_sample, Sampler,
    aaq_resident_workspace_size, aaq_resident_create, aaq_resident_execute, aaq_resident_destroy, Resident,
    aaq_set_half_state, aaq_get_half_state, aaq_energy_grad_noalloc,
)
