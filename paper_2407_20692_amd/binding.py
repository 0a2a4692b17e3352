"""ctypes binding of ``libcpi.so`` (the C ABI in ``include/cpi.h``).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the computation runs in the library's kernels.  The
binding checks dtype, device, contiguity and size of every buffer before a
call, because the C ABI takes bare pointers.  If the library has not been
built, importing this module raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpi.so")

# status codes
OK = 0
ERR_INVALID_ARG = 1
ERR_UNSUPPORTED = 2
ERR_OVERFLOW = 3
ERR_WORKSPACE = 4
ERR_DEVICE = 5
ERR_NOT_READY = 6

FRAMES_U8 = 0
FRAMES_BIT1 = 1
GAMMA_VIEW_MAJOR = 0
GAMMA_PIXEL_MAJOR = 1
MMA_AUTO = 0
MMA_INT8 = 1


class CpiError(RuntimeError):
    def __init__(self, status: int, name: str, detail: str):
        super().__init__(f"{name}: {detail}")
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [
        ("wa", c_int32), ("ha", c_int32), ("wb", c_int32), ("hb", c_int32),
        ("mag_x", c_double), ("mag_y", c_double),
        ("ca_x", c_double), ("ca_y", c_double), ("cb_x", c_double), ("cb_y", c_double),
        ("out_w", c_int32), ("out_h", c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RefocusTiles(ctypes.Structure):
    _fields_ = [("planes_per_group", c_int32), ("rows_per_wave", c_int32),
                ("view_splits", c_int32), ("kernel", c_int32), ("stages", c_int32)]

    def as_tuple(self):
        return (self.planes_per_group, self.rows_per_wave, self.view_splits, self.kernel,
                self.stages)


REFOCUS_ROWS = 0
REFOCUS_COLUMN_SUMS = 1
REFOCUS_VIEW_ROWS = 2


class LensSampling(ctypes.Structure):
    """Lens-plane sample grid (cpi_lens_sampling): x_b = ox + i sx, i < nx;
    y_b = oy + j sy, j < ny."""
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("ox", c_double), ("oy", c_double),
                ("sx", c_double), ("sy", c_double)]


class SideBySide(ctypes.Structure):
    """Raw sensor frames with both detectors side by side (cpi_sidebyside):
    frame_w x frame_h 1-bit pixels, the region roi_w x roi_h at (roi_x, roi_y)
    taken from the left half (detector A) and the right half (detector B)."""
    _fields_ = [
        ("frame_w", c_int32), ("frame_h", c_int32),
        ("roi_x", c_int32), ("roi_y", c_int32), ("roi_w", c_int32), ("roi_h", c_int32),
    ]

    @property
    def frame_bytes(self) -> int:
        return (self.frame_w * self.frame_h + 7) // 8

    @property
    def roi_pixels(self) -> int:
        return self.roi_w * self.roi_h


_SIGS = {
    "cpi_version": (c_char_p, []),
    "cpi_status_string": (c_char_p, [c_int]),
    "cpi_last_error": (c_char_p, []),
    "cpi_geometry_default": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(Geometry)]),
    "cpi_correlate_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "cpi_correlate": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int, c_int,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_size_t, c_void_p]),
    "cpi_correlate_f32_plain_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int,
                                                       POINTER(c_size_t)]),
    "cpi_correlate_f32_plain": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int,
                                        c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "cpi_refocus_workspace_size": (c_int, [POINTER(Geometry), c_int32, POINTER(c_size_t)]),
    "cpi_refocus": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32, c_void_p,
                            c_void_p, c_size_t, c_void_p]),
    "cpi_refocus_plain": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                  c_void_p, c_void_p, c_size_t, c_void_p]),
    "cpi_refocus_noalloc": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                    c_void_p, c_void_p]),
    "cpi_autotune_refocus": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                     c_void_p, c_void_p, c_size_t, c_void_p]),
    "cpi_refocus_config": (c_int, [POINTER(Geometry), c_int32, POINTER(c_int32), POINTER(c_int32),
                                   POINTER(c_int32)]),
    "cpi_refocus_get_tiles": (c_int, [POINTER(Geometry), c_int32, POINTER(RefocusTiles)]),
    "cpi_refocus_tiled": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                  c_void_p, POINTER(RefocusTiles), c_void_p, c_size_t,
                                  c_void_p]),
    "cpi_stream_workspace_size": (c_int, [c_int64, c_int64, c_int, c_int64, POINTER(c_size_t)]),
    "cpi_stream_workspace_size_ex": (c_int, [c_int64, c_int64, c_int, c_int64, c_int32,
                                             POINTER(c_size_t)]),
    "cpi_stream_create_ex": (c_int, [c_int64, c_int64, c_int, c_int64, c_int32, c_void_p,
                                     c_size_t, c_void_p, POINTER(c_void_p)]),
    "cpi_stream_create": (c_int, [c_int64, c_int64, c_int, c_int64, c_void_p, c_size_t, c_void_p,
                                  POINTER(c_void_p)]),
    "cpi_stream_push": (c_int, [c_void_p, c_void_p, c_void_p, c_int64]),
    "cpi_stream_push_host": (c_int, [c_void_p, c_void_p, c_void_p, c_int64]),
    "cpi_stream_frames": (c_int, [c_void_p, POINTER(c_int64)]),
    "cpi_stream_gamma": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p]),
    "cpi_stream_gamma_f32_ptr": (c_int, [c_void_p, POINTER(c_void_p)]),
    "cpi_stream_refocus": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                   c_void_p, c_void_p, c_size_t]),
    "cpi_stream_refocus_async": (c_int, [c_void_p, POINTER(Geometry), POINTER(c_double), c_int32,
                                         c_void_p, c_void_p, c_size_t, c_void_p]),
    "cpi_stream_state_size": (c_int, [c_void_p, POINTER(c_size_t)]),
    "cpi_stream_save": (c_int, [c_void_p, c_void_p, c_size_t]),
    "cpi_stream_load": (c_int, [c_void_p, c_void_p, c_size_t]),
    "cpi_stream_destroy": (c_int, [c_void_p]),
    "cpi_profile_begin": (c_int, []),
    "cpi_profile_end": (c_int, []),
    "cpi_profile_query": (c_int, [c_char_p, POINTER(c_int64), POINTER(c_double)]),
    "cpi_set_mma_encoding": (c_int, [c_int]),
    "cpi_measure_peaks_scratch_size": (c_int, [c_size_t, POINTER(c_size_t)]),
    "cpi_measure_peaks": (c_int, [c_void_p, c_size_t, c_size_t, POINTER(c_double),
                                  POINTER(c_double), POINTER(c_double), c_void_p]),
    "cpi_split_sidebyside": (c_int, [c_void_p, c_int64, POINTER(SideBySide), c_void_p, c_void_p,
                                     c_void_p]),
    "cpi_file_frames": (c_int, [c_char_p, POINTER(SideBySide), POINTER(c_int64)]),
    "cpi_stream_ingest_files": (c_int, [c_void_p, POINTER(c_char_p), c_int32, POINTER(SideBySide),
                                        c_void_p, c_void_p, c_size_t, c_void_p, c_size_t,
                                        POINTER(c_int64)]),
    "cpi_get_mma_encoding": (c_int, []),
    "cpi_lens_sampling_geometry": (c_int, [POINTER(Geometry), POINTER(LensSampling),
                                           POINTER(Geometry)]),
    "cpi_resample_views": (c_int, [c_void_p, POINTER(Geometry), POINTER(LensSampling), c_void_p,
                                   c_void_p]),
    "cpi_refocus_resampled_workspace_size": (c_int, [POINTER(Geometry), POINTER(LensSampling),
                                                     c_int32, POINTER(c_size_t)]),
    "cpi_refocus_resampled": (c_int, [c_void_p, POINTER(Geometry), POINTER(LensSampling),
                                      POINTER(c_double), c_int32, c_void_p, c_void_p, c_size_t,
                                      c_void_p]),
    "cpi_denoiser_layer_count": (c_int, [POINTER(c_int32)]),
    "cpi_denoiser_layer_info": (c_int, [c_int32, c_void_p]),
    "cpi_denoiser_param_count": (c_int, [POINTER(c_int64)]),
    "cpi_denoiser_workspace_size": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "cpi_denoiser_forward": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
    "cpi_denoiser_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float,
                                        c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_size_t, c_void_p]),
    "cpi_denoiser_gradients": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "cpi_image_quality": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                  c_void_p, c_void_p]),
    "cpi_nn_pack_weights": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                    c_void_p]),
    "cpi_nn_conv2d": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                              c_int32, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                              c_void_p]),
    "cpi_nn_conv2d_wgrad_workspace_size": (c_int, [c_int32, c_int32, c_int32, c_int32, c_int32,
                                                   c_int32, POINTER(c_size_t)]),
    "cpi_nn_conv2d_wgrad": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                    c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                    c_void_p]),
    "cpi_nn_upsample2_concat": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                        c_int32, c_void_p, c_void_p]),
    "cpi_nn_upsample2_concat_grad": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32,
                                             c_void_p, c_void_p, c_void_p, c_void_p]),
    "cpi_nn_bias_grad": (c_int, [c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "cpi_nn_maxpool2": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "cpi_nn_maxpool2_grad": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                     c_void_p, c_void_p]),
    "cpi_nn_upsample2": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p,
                                 c_void_p]),
    "cpi_nn_upsample2_grad": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p,
                                      c_void_p, c_void_p]),
    "cpi_nn_concat": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p]),
    "cpi_nn_split": (c_int, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "cpi_nn_add_mask": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "cpi_nn_mse": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                           c_void_p]),
    "cpi_nn_adam": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int64,
                            ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            c_void_p]),
}

EXPORTED = tuple(_SIGS)


def _load():
    # torch ships its own HIP runtime and loads it under a different file name
    # than the soname libcpi.so asks for; importing torch first makes libcpi.so
    # bind to that same runtime instead of starting a second one in the process.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2407_20692_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def version() -> str:
    return lib.cpi_version().decode()


def last_error() -> str:
    return lib.cpi_last_error().decode()


def _check(status: int):
    if status != OK:
        name = lib.cpi_status_string(status).decode()
        raise CpiError(status, name, last_error())


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch  # local: the CPU-only tests load the library without torch work
    return torch


def _dev_ptr(t, what: str, dtype=None, numel: int | None = None, nbytes: int | None = None):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {numel}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return c_void_p(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def frame_bytes(npix: int, fmt: int) -> int:
    return npix if fmt == FRAMES_U8 else (npix + 7) // 8


def _alphas(alphas):
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(POINTER(c_double)), int(a.size)


def alloc_workspace(nbytes: int, device=None):
    """Device workspace as a uint8 tensor (at least 256 bytes)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


# ---------------------------------------------------------------------------
# correlation
# ---------------------------------------------------------------------------

def correlate_workspace_size(n: int, pa: int, pb: int, fmt: int) -> int:
    out = c_size_t(0)
    _check(lib.cpi_correlate_workspace_size(n, pa, pb, fmt, ctypes.byref(out)))
    return out.value


def correlate(frames_a, frames_b, n: int, pa: int, pb: int, fmt: int,
              layout: int = GAMMA_VIEW_MAJOR, gamma=None, gamma_f32=None, numer=None,
              sum_a=None, sum_b=None, workspace=None, stream=None):
    """Exact Gamma of Eq. (1) into the given device tensors (see cpi_correlate).

    A given workspace smaller than correlate_workspace_size makes the library
    work in blocks of frames that fit it (or report CPI_ERR_WORKSPACE)."""
    torch = _torch()
    if workspace is None:
        workspace = alloc_workspace(correlate_workspace_size(n, pa, pb, fmt), frames_a.device)
    have = workspace.numel() * workspace.element_size()
    _check(lib.cpi_correlate(
        _dev_ptr(frames_a, "frames_a", torch.uint8, nbytes=n * frame_bytes(pa, fmt)),
        _dev_ptr(frames_b, "frames_b", torch.uint8, nbytes=n * frame_bytes(pb, fmt)),
        n, pa, pb, fmt, layout,
        _dev_ptr(gamma, "gamma", torch.float64, numel=pa * pb),
        _dev_ptr(gamma_f32, "gamma_f32", torch.float32, numel=pa * pb),
        _dev_ptr(numer, "numer", torch.int64, numel=pa * pb),
        _dev_ptr(sum_a, "sum_a", torch.int64, numel=pa),
        _dev_ptr(sum_b, "sum_b", torch.int64, numel=pb),
        _dev_ptr(workspace, "workspace", torch.uint8), have, _stream(stream)))
    return workspace


def correlate_f32_plain_workspace_size(n: int, pa: int, pb: int, fmt: int) -> int:
    out = c_size_t(0)
    _check(lib.cpi_correlate_f32_plain_workspace_size(n, pa, pb, fmt, ctypes.byref(out)))
    return out.value


def correlate_f32_plain(frames_a, frames_b, n: int, pa: int, pb: int, fmt: int, gamma_f32,
                        layout: int = GAMMA_VIEW_MAJOR, workspace=None, stream=None):
    """Plain FP32 Gamma (see cpi_correlate_f32_plain)."""
    torch = _torch()
    need = correlate_f32_plain_workspace_size(n, pa, pb, fmt)
    if workspace is None:
        workspace = alloc_workspace(need, frames_a.device)
    _check(lib.cpi_correlate_f32_plain(
        _dev_ptr(frames_a, "frames_a", torch.uint8, nbytes=n * frame_bytes(pa, fmt)),
        _dev_ptr(frames_b, "frames_b", torch.uint8, nbytes=n * frame_bytes(pb, fmt)),
        n, pa, pb, fmt, layout,
        _dev_ptr(gamma_f32, "gamma_f32", torch.float32, numel=pa * pb),
        _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need, _stream(stream)))
    return workspace


# ---------------------------------------------------------------------------
# refocus
# ---------------------------------------------------------------------------

def geometry_default(wa: int, ha: int, wb: int, hb: int) -> Geometry:
    g = Geometry()
    _check(lib.cpi_geometry_default(wa, ha, wb, hb, ctypes.byref(g)))
    return g


def make_geometry(**kw) -> Geometry:
    g = Geometry()
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def refocus_workspace_size(g: Geometry, n_alpha: int) -> int:
    out = c_size_t(0)
    _check(lib.cpi_refocus_workspace_size(ctypes.byref(g), n_alpha, ctypes.byref(out)))
    return out.value


def _refocus_call(fn, gamma, g: Geometry, alphas, out, workspace, stream):
    torch = _torch()
    a, ap, na = _alphas(alphas)
    need = refocus_workspace_size(g, na)
    if workspace is None:
        workspace = alloc_workspace(need, gamma.device)
    pa = g.wa * g.ha
    pb = g.wb * g.hb
    _check(fn(_dev_ptr(gamma, "gamma", torch.float32, numel=pa * pb), ctypes.byref(g), ap, na,
              _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h),
              _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need, _stream(stream)))
    del a
    return workspace


def refocus(gamma, g: Geometry, alphas, out, workspace=None, stream=None):
    """Batched refocus of view-major FP32 Gamma into out (n_alpha, out_h, out_w)."""
    return _refocus_call(lib.cpi_refocus, gamma, g, alphas, out, workspace, stream)


def refocus_noalloc(gamma, g: Geometry, alphas, out, stream=None):
    """Batched refocus whose workspace is the library's fixed per-device array
    (no allocation by the library or here); calls on one device must not
    overlap."""
    torch = _torch()
    a, ap, na = _alphas(alphas)
    pa = g.wa * g.ha
    pb = g.wb * g.hb
    _check(lib.cpi_refocus_noalloc(
        _dev_ptr(gamma, "gamma", torch.float32, numel=pa * pb), ctypes.byref(g), ap, na,
        _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h), _stream(stream)))
    del a


def refocus_plain(gamma, g: Geometry, alphas, out, workspace=None, stream=None):
    """One-plane-per-launch refocus (the comparison path)."""
    return _refocus_call(lib.cpi_refocus_plain, gamma, g, alphas, out, workspace, stream)


def lens_sampling(nx: int, ny: int, ox: float, oy: float, sx: float, sy: float) -> LensSampling:
    return LensSampling(nx, ny, ox, oy, sx, sy)


def lens_sampling_geometry(g: Geometry, s: LensSampling) -> Geometry:
    """Geometry under which the resampled views refocus as the sample grid."""
    out = Geometry()
    _check(lib.cpi_lens_sampling_geometry(ctypes.byref(g), ctypes.byref(s), ctypes.byref(out)))
    return out


def resample_views(gamma, g: Geometry, s: LensSampling, views=None, stream=None):
    """FP32 views [ny * nx, Pa] of gamma (FP32 view-major) at the sample grid."""
    torch = _torch()
    pa = g.wa * g.ha
    if views is None:
        views = torch.empty(s.nx * s.ny * pa, dtype=torch.float32, device=gamma.device)
    _check(lib.cpi_resample_views(
        _dev_ptr(gamma, "gamma", torch.float32, numel=pa * g.wb * g.hb), ctypes.byref(g),
        ctypes.byref(s), _dev_ptr(views, "views", torch.float32, numel=s.nx * s.ny * pa),
        _stream(stream)))
    return views


def refocus_resampled_workspace_size(g: Geometry, s: LensSampling, n_alpha: int) -> int:
    out = c_size_t(0)
    _check(lib.cpi_refocus_resampled_workspace_size(ctypes.byref(g), ctypes.byref(s), n_alpha,
                                                    ctypes.byref(out)))
    return out.value


def refocus_resampled(gamma, g: Geometry, s: LensSampling, alphas, out, workspace=None,
                      stream=None):
    torch = _torch()
    a, ap, na = _alphas(alphas)
    need = refocus_resampled_workspace_size(g, s, na)
    if workspace is None:
        workspace = alloc_workspace(need, gamma.device)
    _check(lib.cpi_refocus_resampled(
        _dev_ptr(gamma, "gamma", torch.float32, numel=g.wa * g.ha * g.wb * g.hb), ctypes.byref(g),
        ctypes.byref(s), ap, na, _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h),
        _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need, _stream(stream)))
    del a
    return workspace


def refocus_config(g: Geometry, n_alpha: int):
    """(planes per work-group, rows per wave, view splits) used by refocus()."""
    kp, rw, sp = c_int32(0), c_int32(0), c_int32(0)
    _check(lib.cpi_refocus_config(ctypes.byref(g), n_alpha, ctypes.byref(kp), ctypes.byref(rw),
                                  ctypes.byref(sp)))
    return kp.value, rw.value, sp.value


def refocus_tiles(g: Geometry, n_alpha: int):
    """(planes per work-group, rows per wave, view splits, kernel, stages) used by
    refocus()."""
    t = RefocusTiles()
    _check(lib.cpi_refocus_get_tiles(ctypes.byref(g), n_alpha, ctypes.byref(t)))
    return t.as_tuple()


def refocus_tiled(gamma, g: Geometry, alphas, out, tiles, workspace=None, stream=None):
    """Batched refocus with an explicit configuration (planes per work-group,
    rows per wave, view splits, kernel[, stages]); stages default to 3."""
    vals = [int(v) for v in tiles]
    if len(vals) == 4:
        vals.append(3)
    t = RefocusTiles(*vals)
    torch = _torch()
    a, ap, na = _alphas(alphas)
    need = refocus_workspace_size(g, na)
    if workspace is None:
        workspace = alloc_workspace(need, gamma.device)
    pa = g.wa * g.ha
    pb = g.wb * g.hb
    _check(lib.cpi_refocus_tiled(
        _dev_ptr(gamma, "gamma", torch.float32, numel=pa * pb), ctypes.byref(g), ap, na,
        _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h), ctypes.byref(t),
        _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need, _stream(stream)))
    del a
    return workspace


def autotune_refocus(gamma, g: Geometry, alphas, out, workspace=None, stream=None):
    """Times the refocus configurations, caches the best, leaves the result in out."""
    return _refocus_call(lib.cpi_autotune_refocus, gamma, g, alphas, out, workspace, stream)


def set_mma_encoding(enc: int):
    """MMA_AUTO (FP4 operands for binary frames where exact) or MMA_INT8;
    process-wide, for calls enqueued afterwards."""
    _check(lib.cpi_set_mma_encoding(enc))


def get_mma_encoding() -> int:
    return lib.cpi_get_mma_encoding()


def measure_peaks(device=None, copy_bytes: int = 1 << 30, stream=None):
    """Measured int8 and FP4 matrix-core ops/s and device-copy bytes/s
    (read + write) of the current device."""
    torch = _torch()
    need = c_size_t(0)
    _check(lib.cpi_measure_peaks_scratch_size(copy_bytes, ctypes.byref(need)))
    scratch = alloc_workspace(need.value, device)
    i8, f4, bw = c_double(0), c_double(0), c_double(0)
    _check(lib.cpi_measure_peaks(_dev_ptr(scratch, "scratch", torch.uint8), need.value, copy_bytes,
                                 ctypes.byref(i8), ctypes.byref(f4), ctypes.byref(bw),
                                 _stream(stream)))
    return {"int8_ops_per_s": i8.value, "fp4_ops_per_s": f4.value, "copy_bytes_per_s": bw.value}


# ---------------------------------------------------------------------------
# raw side-by-side sensor frames
# ---------------------------------------------------------------------------

def sidebyside(frame_w: int, frame_h: int, roi_x: int = 0, roi_y: int = 0, roi_w: int = None,
               roi_h: int = None) -> SideBySide:
    """Layout of raw frames; the region defaults to the whole half frame."""
    return SideBySide(frame_w, frame_h, roi_x, roi_y,
                      frame_w // 2 if roi_w is None else roi_w,
                      frame_h if roi_h is None else roi_h)


def split_sidebyside(frames, n: int, f: SideBySide, out_a, out_b, stream=None):
    """n raw frames (device uint8) -> 1-bit frames of both detectors' regions."""
    torch = _torch()
    ob = n * ((f.roi_pixels + 7) // 8)
    _check(lib.cpi_split_sidebyside(
        _dev_ptr(frames, "frames", torch.uint8, nbytes=n * f.frame_bytes), n, ctypes.byref(f),
        _dev_ptr(out_a, "out_a", torch.uint8, nbytes=ob),
        _dev_ptr(out_b, "out_b", torch.uint8, nbytes=ob), _stream(stream)))


def file_frames(path: str, f: SideBySide) -> int:
    """Whole raw frames in a file (host only)."""
    n = c_int64(0)
    _check(lib.cpi_file_frames(os.fsencode(path), ctypes.byref(f), ctypes.byref(n)))
    return n.value


# ---------------------------------------------------------------------------
# kernel timing
# ---------------------------------------------------------------------------

def profile_begin():
    _check(lib.cpi_profile_begin())


def profile_end():
    _check(lib.cpi_profile_end())


def profile_query(group: str):
    """(launches, total milliseconds) recorded for one kernel group."""
    n = c_int64(0)
    ms = c_double(0.0)
    _check(lib.cpi_profile_query(group.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ---------------------------------------------------------------------------
# streaming
# ---------------------------------------------------------------------------

def stream_workspace_size(pa: int, pb: int, fmt: int, max_chunk: int,
                          gamma_buffers: int = 1) -> int:
    out = c_size_t(0)
    _check(lib.cpi_stream_workspace_size_ex(pa, pb, fmt, max_chunk, gamma_buffers,
                                            ctypes.byref(out)))
    return out.value


class Stream:
    """Device-resident running sums of Eq. (1), updated chunk by chunk.
    gamma_buffers=2 keeps two FP32 Gamma buffers so that refocus_async of
    chunk k (on another stream) overlaps the update of chunk k + 1."""

    def __init__(self, pa: int, pb: int, fmt: int, max_chunk: int, device=None, stream=None,
                 gamma_buffers: int = 1):
        torch = _torch()
        self.pa, self.pb, self.fmt, self.max_chunk = pa, pb, fmt, max_chunk
        need = stream_workspace_size(pa, pb, fmt, max_chunk, gamma_buffers)
        self.workspace = alloc_workspace(need, device)
        self._stream = stream
        h = c_void_p()
        _check(lib.cpi_stream_create_ex(pa, pb, fmt, max_chunk, gamma_buffers,
                                        _dev_ptr(self.workspace, "workspace", torch.uint8,
                                                 nbytes=need),
                                        need, _stream(stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.cpi_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, chunk_a, chunk_b, k: int):
        torch = _torch()
        _check(lib.cpi_stream_push(
            self.handle,
            _dev_ptr(chunk_a, "chunk_a", torch.uint8, nbytes=k * frame_bytes(self.pa, self.fmt)),
            _dev_ptr(chunk_b, "chunk_b", torch.uint8, nbytes=k * frame_bytes(self.pb, self.fmt)),
            k))

    def push_host(self, chunk_a, chunk_b, k: int):
        """Host chunks: numpy arrays or CPU tensors (pinned ones copy asynchronously)."""
        keep = []

        def host_ptr(x, nb, what):
            if hasattr(x, "data_ptr"):
                if x.is_cuda or not x.is_contiguous() or x.numel() * x.element_size() < nb:
                    raise ValueError(f"{what} must be a contiguous host buffer of {nb} bytes")
                return c_void_p(x.data_ptr())
            arr = np.ascontiguousarray(x, dtype=np.uint8)
            if arr.nbytes < nb:
                raise ValueError(f"{what} must hold {nb} bytes")
            keep.append(arr)
            return c_void_p(arr.ctypes.data)

        _check(lib.cpi_stream_push_host(
            self.handle,
            host_ptr(chunk_a, k * frame_bytes(self.pa, self.fmt), "chunk_a"),
            host_ptr(chunk_b, k * frame_bytes(self.pb, self.fmt), "chunk_b"), k))
        if keep:
            # pageable memory: the copy is complete before the call returned
            del keep

    def ingest_files(self, paths, f: SideBySide, host_a, host_b, dev_raw) -> int:
        """Folds every frame of the raw frame files into the sums (host_a,
        host_b: CPU uint8 tensors of equal size, pinned for overlap; dev_raw:
        device uint8 tensor).  Returns the frames ingested; the buffers stay in
        use until the stream has reached the enqueued work."""
        torch = _torch()
        for x, what in ((host_a, "host_a"), (host_b, "host_b")):
            if x.is_cuda or x.dtype != torch.uint8 or not x.is_contiguous():
                raise ValueError(f"{what} must be a contiguous CPU uint8 tensor")
        hb = min(host_a.numel(), host_b.numel())
        arr = (c_char_p * len(paths))(*[os.fsencode(p) for p in paths])
        n = c_int64(0)
        _check(lib.cpi_stream_ingest_files(
            self.handle, arr, len(paths), ctypes.byref(f), c_void_p(host_a.data_ptr()),
            c_void_p(host_b.data_ptr()), hb,
            _dev_ptr(dev_raw, "dev_raw", torch.uint8), dev_raw.numel(), ctypes.byref(n)))
        return n.value

    @property
    def frames(self) -> int:
        n = c_int64(0)
        _check(lib.cpi_stream_frames(self.handle, ctypes.byref(n)))
        return n.value

    def gamma(self, layout: int = GAMMA_VIEW_MAJOR, gamma=None, gamma_f32=None, numer=None,
              sum_a=None, sum_b=None):
        torch = _torch()
        n = self.pa * self.pb
        _check(lib.cpi_stream_gamma(
            self.handle, layout,
            _dev_ptr(gamma, "gamma", torch.float64, numel=n),
            _dev_ptr(gamma_f32, "gamma_f32", torch.float32, numel=n),
            _dev_ptr(numer, "numer", torch.int64, numel=n),
            _dev_ptr(sum_a, "sum_a", torch.int64, numel=self.pa),
            _dev_ptr(sum_b, "sum_b", torch.int64, numel=self.pb)))

    def gamma_f32_ptr(self) -> int:
        p = c_void_p()
        _check(lib.cpi_stream_gamma_f32_ptr(self.handle, ctypes.byref(p)))
        return p.value

    def refocus(self, g: Geometry, alphas, out, workspace=None):
        torch = _torch()
        a, ap, na = _alphas(alphas)
        need = refocus_workspace_size(g, na)
        if workspace is None:
            workspace = alloc_workspace(need, self.workspace.device)
        _check(lib.cpi_stream_refocus(
            self.handle, ctypes.byref(g), ap, na,
            _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h),
            _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need))
        del a
        return workspace

    def refocus_async(self, g: Geometry, alphas, out, workspace, stream):
        """Refocus of the latest push's Gamma enqueued on `stream` (after that
        push); out and workspace stay in use until `stream` reaches it."""
        torch = _torch()
        a, ap, na = _alphas(alphas)
        need = refocus_workspace_size(g, na)
        _check(lib.cpi_stream_refocus_async(
            self.handle, ctypes.byref(g), ap, na,
            _dev_ptr(out, "out", torch.float32, numel=na * g.out_w * g.out_h),
            _dev_ptr(workspace, "workspace", torch.uint8, nbytes=need), need, _stream(stream)))
        del a

    def state_size(self) -> int:
        out = c_size_t(0)
        _check(lib.cpi_stream_state_size(self.handle, ctypes.byref(out)))
        return out.value

    def save(self) -> bytes:
        buf = ctypes.create_string_buffer(self.state_size())
        _check(lib.cpi_stream_save(self.handle, buf, len(buf)))
        return buf.raw

    def load(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        _check(lib.cpi_stream_load(self.handle, buf, len(state)))
