"""FP64 CPU reference oracle for the soft-shadow hot path (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg (``cpu_baseline`` and the host timings beside it, skipped with ``--no-cpu``)
may import this package.  It shares no code with the HIP library and never
reads anything the GPU path produced.

The numerics live in plain C (``oracle.c``, ``alternatives.c``, ``view.c``, ``resample.c``), compiled with
gcc into ``liboracle.so`` and called through ctypes; the reference gradient is
torch float64 autograd (``grad_ref.py``).
"""
from .core import (  # noqa: F401
    Params, build, load, maxmip_levels, maxmip, shadow, shadow_threaded, shadow_points,
    alternatives,
    disc_fraction, schedule, ray_consts, probe, path_cells, tap_bound, TRACE_DTYPE,
    Camera, ViewTol, VIEW_DTYPE, view, view_threaded, view_direction, view_probe,
    Frame, resample, frame_source_coords,
)
