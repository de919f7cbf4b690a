"""MI355X-native soft shadows on planetary heightfields (dynamic programming over
a maximum mipmap).  The compute runs in libsoftshadow.so (HIP, gfx950); this
package only marshals torch tensors into its C ABI (include/softshadow.h).
"""
from .api import (  # noqa: F401
    Params, maxmip, maxmip_levels, maxmip_floats, maxmip_level_offset, maxmip_unpack,
    shadow_cast, shadow_cast_counted, shadow_cast_backward, shadow, ShadowCast,
    shadow_cast_batched, batched_workspace_bytes, BatchedPlan, SUN_RADIUS_RAD,
    bound_build, bound_floats, bound_level_offset, bound_unpack,
    shadow_cast_save, shadow_cast_backward_saved, shadow_cast_backward_penumbra, probe_gather,
    probe_gather_tiles, probe_valu, shadow_points,
    Camera, view_cast, frame, Frame, resample, stitch, shadow_points_image,
    shadow_points_backward, ShadowPoints, shadow_at,
)
from ._lib import lib, SoftShadowError, RAY_TILES, SS_MODE_DP, SS_MODE_UNIFORM  # noqa: F401
from ._lib import SS_MODE_EXACT, SS_MODE_POINT, SS_VIEW_HIER, SS_VIEW_DENSE  # noqa: F401
from ._lib import SS_SCHED_EQUAL, SS_SCHED_GEOMETRIC, SS_SCHED_LIST  # noqa: F401
