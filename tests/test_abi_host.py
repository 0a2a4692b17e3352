"""The C ABI library loads on a host without a GPU, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpi.h")


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpi_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(cpi):
    syms = declared_symbols()
    assert len(syms) >= 24
    lib = ctypes.CDLL(cpi.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(cpi.EXPORTED)


def test_version_and_status_strings(cpi):
    assert "gfx950" in cpi.version()
    assert cpi.lib.cpi_status_string(0) == b"CPI_OK"
    assert cpi.lib.cpi_status_string(4) == b"CPI_ERR_WORKSPACE"


def test_workspace_sizes(cpi):
    s1 = cpi.correlate_workspace_size(1000, 1024, 256, cpi.FRAMES_U8)
    s2 = cpi.correlate_workspace_size(1000, 1024, 256, cpi.FRAMES_BIT1)
    assert s1 > s2 > 0
    # U8 above 131008 frames needs the int64 accumulator of the flush passes
    big = cpi.correlate_workspace_size(140000, 64, 32, cpi.FRAMES_U8)
    assert big >= 64 * 32 * 8 + 96 * 140032
    # past one ingest pass (2^24 - 512 frames; reachable for 1-bit frames, as
    # byte frames overflow int64 first) the frames are folded in blocks of
    # that many frames: the workspace no longer grows with n
    one_pass = (1 << 24) - 512
    last = cpi.correlate_workspace_size(one_pass, 40, 24, cpi.FRAMES_BIT1)
    past = cpi.correlate_workspace_size(one_pass + 1, 40, 24, cpi.FRAMES_BIT1)
    assert past == cpi.correlate_workspace_size(1 << 25, 40, 24, cpi.FRAMES_BIT1) > 0
    assert past <= 2 * last
    assert cpi.correlate_f32_plain_workspace_size(20000, 16384, 4096, cpi.FRAMES_U8) >= \
        20000 * (16384 + 4096) * 4
    g = cpi.geometry_default(128, 128, 64, 64)
    assert cpi.refocus_workspace_size(g, 32) >= 32 * (128 + 128 + 64 + 64) * 8
    assert cpi.stream_workspace_size(16384, 4096, cpi.FRAMES_BIT1, 1000) >= 16384 * 4096 * 8
    # chunks are limited to one ingest pass (1-bit) and one int32 pass (bytes)
    assert cpi.stream_workspace_size(64, 32, cpi.FRAMES_BIT1, (1 << 24) - 512) > 0
    assert cpi.stream_workspace_size(64, 32, cpi.FRAMES_U8, 131008) > 0
    for fmt, chunk in ((cpi.FRAMES_BIT1, (1 << 24) - 511), (cpi.FRAMES_U8, 131009)):
        with pytest.raises(cpi.CpiError) as e:
            cpi.stream_workspace_size(64, 32, fmt, chunk)
        assert e.value.status == 1


@pytest.mark.parametrize("args,status", [
    ((0, 10, 10, 0), 1),
    ((10, 0, 10, 0), 1),
    ((10, 10, -1, 1), 1),
    ((10, 10, 10, 7), 1),
    ((11_909_806, 1, 1, 0), 3),           # u8 int64 bound
    ((11_909_805, 1, 1, 0), 0),
    ((94_906_266, 1, 1, 1), 3),           # N^2 >= 2^53
    ((94_906_265, 1, 1, 1), 0),
    ((1 << 20, 1 << 21, 1 << 20, 1), 1),  # Pa * Pb too large
])
def test_correlate_validation(cpi, args, status):
    out = ctypes.c_size_t(0)
    assert cpi.lib.cpi_correlate_workspace_size(*args, ctypes.byref(out)) == status


def test_correlate_rejects_before_launch(cpi):
    lib = cpi.lib
    # null frames, misaligned frames, no outputs, small workspace: all host-side
    fake = ctypes.c_void_p(0x10000)
    mis = ctypes.c_void_p(0x10008)
    assert lib.cpi_correlate(None, fake, 10, 10, 10, 0, 0, fake, None, None, None, None,
                             fake, 1 << 30, None) == 1
    assert lib.cpi_correlate(mis, fake, 10, 10, 10, 0, 0, fake, None, None, None, None,
                             fake, 1 << 30, None) == 1
    assert lib.cpi_correlate(fake, fake, 10, 10, 10, 0, 0, None, None, None, None, None,
                             fake, 1 << 30, None) == 1
    assert lib.cpi_correlate(fake, fake, 10, 10, 10, 0, 5, fake, None, None, None, None,
                             fake, 1 << 30, None) == 1
    assert lib.cpi_correlate(fake, fake, 10, 10, 10, 0, 0, fake, None, None, None, None,
                             fake, 16, None) == 4
    assert "workspace" in cpi.last_error()


def test_refocus_validation(cpi):
    lib = cpi.lib
    g = cpi.geometry_default(32, 32, 16, 16)
    fake = ctypes.c_void_p(0x10000)
    al = (ctypes.c_double * 2)(0.5, float("nan"))
    assert lib.cpi_refocus(fake, ctypes.byref(g), al, 2, fake, fake, 1 << 30, None) == 1
    assert "finite" in cpi.last_error()
    al = (ctypes.c_double * 1)(1.0)
    assert lib.cpi_refocus(fake, ctypes.byref(g), al, 0, fake, fake, 1 << 30, None) == 1
    assert lib.cpi_refocus(fake, ctypes.byref(g), al, 1, fake, fake, 8, None) == 4
    bad = cpi.geometry_default(32, 32, 16, 16)
    bad.mag_x = float("inf")
    assert lib.cpi_refocus(fake, ctypes.byref(bad), al, 1, fake, fake, 1 << 30, None) == 1
    bad = cpi.geometry_default(32, 32, 16, 16)
    bad.out_w = 0
    assert lib.cpi_refocus(fake, ctypes.byref(bad), al, 1, fake, fake, 1 << 30, None) == 1
    huge = (ctypes.c_double * 1)(1e12)
    assert lib.cpi_refocus(fake, ctypes.byref(g), huge, 1, fake, fake, 1 << 30, None) == 1
    # explicit configurations: a null one is invalid, an unbuilt one unsupported
    # (CPI_ERR_UNSUPPORTED = 2), both before any launch; argument checks as above
    assert lib.cpi_refocus_tiled(fake, ctypes.byref(g), al, 1, fake, None, fake, 1 << 30,
                                 None) == 1
    for t in [(2, 8, 1, 0, 0), (8, 16, 1, 1, 1), (8, 32, 1, 1, 4), (8, 16, 0, 0, 0),
              (8, 16, 17, 1, 2), (1, 16, 1, 0, 0)]:
        tiles = cpi.RefocusTiles(*t)
        assert lib.cpi_refocus_tiled(fake, ctypes.byref(g), al, 1, fake, ctypes.byref(tiles),
                                     fake, 1 << 30, None) == 2, t
    tiles = cpi.RefocusTiles(4, 16, 2, 1, 2)
    assert lib.cpi_refocus_tiled(fake, ctypes.byref(g), al, 0, fake, ctypes.byref(tiles), fake,
                                 1 << 30, None) == 1
    out = cpi.RefocusTiles()
    assert lib.cpi_refocus_get_tiles(ctypes.byref(g), 5, None) == 1
    assert lib.cpi_refocus_get_tiles(ctypes.byref(g), 5, ctypes.byref(out)) == 0


def test_stream_validation(cpi):
    lib = cpi.lib
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x10000)
    assert lib.cpi_stream_create(64, 16, 1, 0, fake, 1 << 30, None, ctypes.byref(h)) == 1
    assert lib.cpi_stream_create(64, 16, 0, 200000, fake, 1 << 30, None, ctypes.byref(h)) == 1
    assert lib.cpi_stream_create(64, 16, 1, 100, fake, 16, None, ctypes.byref(h)) == 4
    assert lib.cpi_stream_push(None, fake, fake, 1) == 1


def test_default_geometry(cpi):
    g = cpi.geometry_default(128, 96, 64, 32)
    assert (g.mag_x, g.mag_y, g.ca_x, g.ca_y, g.cb_x, g.cb_y) == (2.0, 3.0, 63.5, 47.5, 31.5, 15.5)
    assert (g.out_w, g.out_h) == (128, 96)


def test_mma_encoding_switch(cpi):
    before = cpi.get_mma_encoding()
    try:
        cpi.set_mma_encoding(cpi.MMA_INT8)
        assert cpi.get_mma_encoding() == cpi.MMA_INT8
        cpi.set_mma_encoding(cpi.MMA_AUTO)
        assert cpi.get_mma_encoding() == cpi.MMA_AUTO
        assert cpi.lib.cpi_set_mma_encoding(7) == 1          # CPI_ERR_INVALID_ARG
        assert cpi.get_mma_encoding() == cpi.MMA_AUTO
    finally:
        cpi.set_mma_encoding(before)


def test_denoiser_host_validation(cpi):
    """Layer table, parameter layout and argument checks of the denoiser
    entry points (host logic only, nothing is launched)."""
    import paper_2407_20692_amd.denoiser as dn_lib
    import oracle.denoiser as dn_ref

    infos = dn_lib.layers()
    assert [L.name for L in infos] == [L.name for L in dn_ref.layers()]
    total = dn_lib.param_count()
    end = 0
    for L in infos:
        assert L.weight_offset >= end and L.bias_offset >= L.weight_offset + L.weight_count
        end = L.bias_offset + L.cout
    assert end <= total
    assert dn_lib.workspace_size(16, 128, 128, True) > dn_lib.workspace_size(16, 128, 128, False)
    lib = cpi.lib
    out = ctypes.c_size_t(0)
    assert lib.cpi_denoiser_workspace_size(0, 16, 16, 0, ctypes.byref(out)) == 1
    assert lib.cpi_denoiser_workspace_size(1, 12, 16, 0, ctypes.byref(out)) == 1
    assert lib.cpi_denoiser_workspace_size(1 << 12, 1024, 1024, 0, ctypes.byref(out)) == 1
    fake = ctypes.c_void_p(1 << 20)
    assert lib.cpi_denoiser_forward(fake, 1, 16, 16, fake, fake, fake, 16, None) == 4
    assert lib.cpi_denoiser_train_step(fake, fake, fake, 0, 1e-3, 1, 16, 16, fake, fake, fake,
                                       fake, 1 << 40, None) == 1
    assert lib.cpi_denoiser_train_step(fake, fake, fake, 1, 0.0, 1, 16, 16, fake, fake, fake,
                                       fake, 1 << 40, None) == 1
    # conv channel rules: cin % 8, cout % 32, odd ks, kpad consistent
    assert lib.cpi_nn_conv2d(fake, fake, None, None, 0, 1, 4, 4, 12, 32, 3, 128, fake, None,
                             None) == 1
    assert lib.cpi_nn_conv2d(fake, fake, None, None, 0, 1, 4, 4, 8, 48, 3, 96, fake, None,
                             None) == 1
    assert lib.cpi_nn_conv2d(fake, fake, None, None, 0, 1, 4, 4, 8, 32, 2, 32, fake, None,
                             None) == 1
    assert lib.cpi_nn_conv2d(fake, fake, None, None, 0, 1, 4, 4, 8, 32, 3, 64, fake, None,
                             None) == 1
    assert lib.cpi_nn_maxpool2(fake, 1, 5, 4, 8, fake, None) == 1
    assert lib.cpi_image_quality(fake, fake, 1, 10, 16, fake, fake, None) == 1


def test_resampled_refocus_host_validation(cpi):
    lib = cpi.lib
    g = cpi.geometry_default(16, 16, 8, 8)
    ok = cpi.lens_sampling(15, 15, 0.0, 0.0, 0.5, 0.5)
    gs = cpi.lens_sampling_geometry(g, ok)
    assert (gs.wb, gs.hb, gs.mag_x, gs.cb_x) == (15, 15, 1.0, 7.0)
    need = cpi.refocus_resampled_workspace_size(g, ok, 4)
    assert need >= 15 * 15 * 256 * 4
    out = ctypes.c_size_t(0)
    for bad in (cpi.lens_sampling(0, 3, 0, 0, 1, 1), cpi.lens_sampling(3, 3, 0, 0, 0.0, 1),
                cpi.lens_sampling(3, 3, float("nan"), 0, 1, 1),
                cpi.lens_sampling(3, 3, 0, 0, 1, -2.0)):
        assert lib.cpi_refocus_resampled_workspace_size(ctypes.byref(g), ctypes.byref(bad), 4,
                                                        ctypes.byref(out)) == 1
    fake = ctypes.c_void_p(1 << 20)
    al = (ctypes.c_double * 2)(0.5, 1.0)
    assert lib.cpi_refocus_resampled(fake, ctypes.byref(g), ctypes.byref(ok), al, 2, fake, fake,
                                     16, None) == 4
    assert lib.cpi_resample_views(None, ctypes.byref(g), ctypes.byref(ok), fake, None) == 1


def test_memory_adaptive_workspace_host(cpi):
    """CPI_WORKSPACE_LIMIT lowers the reported correlate workspace to a blocked
    plan that fits, and a workspace below even one 512-frame block is refused
    before anything is launched."""
    import os
    n, pa, pb = 100000, 1024, 1024
    full = cpi.correlate_workspace_size(n, pa, pb, cpi.FRAMES_BIT1)
    os.environ["CPI_WORKSPACE_LIMIT"] = "12000000"
    try:
        lim = cpi.correlate_workspace_size(n, pa, pb, cpi.FRAMES_BIT1)
    finally:
        del os.environ["CPI_WORKSPACE_LIMIT"]
    assert lim <= 12000000 < full
    fake = ctypes.c_void_p(1 << 20)
    st = cpi.lib.cpi_correlate(fake, fake, n, pa, pb, 1, 0, fake, None, None, None, None, fake,
                               4096, None)
    assert st == 4
    assert b"blocks of 512 frames" in cpi.lib.cpi_last_error()


_TILES_SCRIPT = """
import sys
sys.path.insert(0, {root!r})
import paper_2407_20692_amd as cpi
g = cpi.geometry_default(32, 32, 16, 16)
print(*cpi.refocus_tiles(g, 5))
"""


def _tiles_with_cache(tmp_path, lines):
    """refocus_tiles in a fresh process whose autotune cache file holds
    `lines` (the cache is read once per process)."""
    import subprocess
    import sys

    cache = tmp_path / "cache.txt"
    cache.write_text("".join(line + "\n" for line in lines))
    env = dict(os.environ, CPI_AUTOTUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", _TILES_SCRIPT.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=300, check=True)
    return tuple(int(v) for v in r.stdout.split())


def test_autotune_cache_file(tmp_path):
    """A cached configuration (planes per group, rows, view splits, kernel,
    staged windows) is used for its shape; a file with a line in another
    format or naming a configuration that is not built is ignored as a whole,
    leaving the default (column-sum kernel, 4 planes x 16 rows, 2 stages).
    Without a GPU the device part of the key is 'dev?'."""
    key = "wa32_ha32_wb16_hb16_ow32_oh32_na5@dev?"
    assert _tiles_with_cache(tmp_path, [f"{key} 8 8 2 1 3 123.0"]) == (8, 8, 2, 1, 3)
    assert _tiles_with_cache(tmp_path, [f"{key} 16 16 4 0 0 99.5"]) == (16, 16, 4, 0, 0)
    default = _tiles_with_cache(tmp_path, [])
    assert default[:2] == (4, 16) and default[3:] == (1, 2) and 1 <= default[2] <= 16
    # the earlier four-column format, an unbuilt shape, too many stages for LDS
    for bad in [f"{key} 8 8 2 123.0", f"{key} 2 8 1 1 2 5.0", f"{key} 8 32 1 1 4 5.0"]:
        assert _tiles_with_cache(tmp_path, [f"{key} 8 8 2 1 3 1.0", bad]) == default
