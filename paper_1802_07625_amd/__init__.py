"""MI355X (gfx950) hot path of the fast flow-based cartogram method.

One iteration = areas -> density grid -> blur + flux transforms -> adaptive
Dormand-Prince advection of all points -> areas and relative errors, all in
HIP kernels behind the C ABI of include/ffb.h (libffb.so, built in-tree).
"""
from .api import (  # noqa: F401
    Context, Geometry, IntegrateOpts, IterationResult, FFBError, STATUS,
    default_sigma, iterate, lib, LIB_PATH,
    ffb_create, ffb_destroy, ffb_sync, ffb_reset_status, ffb_last_error,
    ffb_area_error, ffb_density, ffb_flux, ffb_pack_fields, ffb_integrate,
    ffb_set_option, OPT_ADVECT_STATE, OPT_ADVECT_BLOCKS, OPT_DIFFUSION_GRAPH, OPT_POINT_ORDER,
    POINT_ORDER_GIVEN, POINT_ORDER_AUTO, POINT_ORDER_ALWAYS, POINT_ORDER_KEEP,
    ffb_diffusion, ffb_diffusion_fields, iterate_diffusion, diffusion_t_end, DIFFUSION_K,
    ffb_area_adj, ffb_density_adj, ffb_flux_adj, ffb_integrate_record, ffb_integrate_adj,
    ffb_tape_begin, ffb_tape_end, ffb_tape_clear, ffb_tape_generation, ffb_tape_check,
    ffb_backward, FFBFunction,
    FFB_OK, FFB_E_INVALID, FFB_E_NOMEM, FFB_E_DEVICE, FFB_E_NONPOSITIVE, FFB_E_DOMAIN,
    FFB_E_STEP_UNDERFLOW, FFB_E_NONFINITE, FFB_E_NO_TAPE, FFB_E_MAX_ATTEMPTS, FFB_E_TOO_LARGE,
    Batch, BatchOpts, ffb_distortion, ffb_inverse,
)
