"""NARVis hot path on MI355X: multi-attribute point rasterizer (HIP, gfx950).

The compute lives in libnarvis.so (built from csrc/ by build.py); this package
holds its Python binding (narvis.py, same entry-point names as the C ABI in
include/narvis.h) and the seeded synthetic workloads (scenes.py).
"""
from .narvis import (GBuffer, NarvisError, RENDER_AUTO, RENDER_EARLYZ, RENDER_GLOBAL,  # noqa: F401
                     narvis_camera_matrix, narvis_raster_clear, narvis_raster_render, narvis_raster_resolve,
                     narvis_rasterize, narvis_status_string, SplatParams, COLOR_LUT, COLOR_RGB8,
                     narvis_splat, narvis_splat_workspace_size)
