"""CPU oracle for correlation plenoptic imaging -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the GPU path
computes, written from the paper's definitions:

* ``correlation``  -- the 4-D correlation function Gamma of Eq. (1)
  (Section "CPI algorithm", item 1), evaluated exactly as an integer numerator
  over N^2;
* ``refocus``      -- shift-and-sum refocusing (Section "CPI algorithm",
  item 2; refocusing optimisation in Section 4.1), one bilinear sample of every
  perspective view per output pixel and plane, summed over views, in FP64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it; the library never imports this package.

Pin status: every function here is pinned by ``-m "not gpu"`` tests against
closed forms, invariants, brute force in exact rational arithmetic and
hand-worked examples (``tests/test_oracle_*.py``); none is "parity unpinned".
"""
from .correlation import (
    FRAMES_U8,
    FRAMES_BIT1,
    GAMMA_VIEW_MAJOR,
    GAMMA_PIXEL_MAJOR,
    frame_bytes,
    unpack_frames,
    correlation,
    to_layout,
    overflow_ok,
)
from .refocus import (Geometry, LensSampling, default_geometry, refocus, refocus_pixels,
                      refocus_resampled, refocus_resampled_pixels)

__all__ = [
    "FRAMES_U8",
    "FRAMES_BIT1",
    "GAMMA_VIEW_MAJOR",
    "GAMMA_PIXEL_MAJOR",
    "frame_bytes",
    "unpack_frames",
    "correlation",
    "to_layout",
    "overflow_ok",
    "Geometry",
    "default_geometry",
    "refocus",
    "refocus_pixels",
    "LensSampling",
    "refocus_resampled",
    "refocus_resampled_pixels",
]
