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
    ffb_set_option, OPT_ADVECT_STATE, OPT_ADVECT_BLOCKS,
)
