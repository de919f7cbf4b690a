"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the soft-shadow method: it only draws
heightfields (fBm plus craters) and sun directions.  Both the FP64 oracle and
the HIP path read the arrays it produces; neither side imports the other.
"""
from .dem import fbm, add_craters, make_dem  # noqa: F401
from .configs import CONFIGS, config, sun_list, dem_for, seed_of, R_MOON, SUN_RADIUS_RAD  # noqa: F401
from .configs import look_at, view_scene  # noqa: F401
from .planet import planet_height, frame_dirs, seam_scene, seam_frames  # noqa: F401
