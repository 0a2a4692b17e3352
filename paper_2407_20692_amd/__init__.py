"""MI355X (gfx950) correlation plenoptic imaging: exact correlation function
and batched refocusing behind the C ABI of ``include/cpi.h``.

Importing the package loads ``libcpi.so``; it raises ImportError when the
library has not been built (``python paper_2407_20692_amd/build.py``).
"""
from .binding import (  # noqa: F401
    CpiError,
    EXPORTED,
    FRAMES_BIT1,
    FRAMES_U8,
    GAMMA_PIXEL_MAJOR,
    GAMMA_VIEW_MAJOR,
    Geometry,
    LIB_PATH,
    MMA_AUTO,
    MMA_INT8,
    Stream,
    alloc_workspace,
    autotune_refocus,
    correlate,
    correlate_f32_plain,
    correlate_f32_plain_workspace_size,
    correlate_workspace_size,
    frame_bytes,
    geometry_default,
    get_mma_encoding,
    last_error,
    lib,
    make_geometry,
    profile_begin,
    profile_end,
    profile_query,
    refocus,
    refocus_config,
    refocus_plain,
    refocus_workspace_size,
    set_mma_encoding,
    stream_workspace_size,
    version,
)
