"""Raw side-by-side frame files on the host: frame counting and rejection of
malformed layouts and files (no device work)."""
import os

import numpy as np
import pytest

from synth import compose_sidebyside, pack_raw_frames, write_frame_files


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def test_compose_and_pack_layout():
    rng = np.random.default_rng(1)
    a = (rng.random((3, 4, 5)) < 0.5).astype(np.uint8)
    b = (rng.random((3, 4, 5)) < 0.5).astype(np.uint8)
    raw = compose_sidebyside(a, b, frame_w=16, frame_h=6, roi_x=2, roi_y=1, rng=rng)
    assert np.array_equal(raw[:, 1:5, 2:7], a) and np.array_equal(raw[:, 1:5, 10:15], b)
    packed = pack_raw_frames(raw)
    assert packed.shape == (3, 12)
    # pixel (y, x) is bit (y*16 + x) % 8 of byte (y*16 + x) // 8
    y, x = 3, 11
    bit = y * 16 + x
    assert (packed[2, bit // 8] >> (bit % 8)) & 1 == raw[2, y, x]


def test_file_frames(cpi, tmp_path):
    f = cpi.sidebyside(64, 24)
    raw = np.zeros((10, 24, 64), np.uint8)
    paths = write_frame_files(str(tmp_path), pack_raw_frames(raw), [7, 3])
    assert [cpi.file_frames(p, f) for p in paths] == [7, 3]
    with open(paths[1], "ab") as fh:
        fh.write(b"\0")
    with pytest.raises(cpi.CpiError) as e:
        cpi.file_frames(paths[1], f)
    assert e.value.status == 1 and "whole number" in str(e.value)
    with pytest.raises(cpi.CpiError):
        cpi.file_frames(os.path.join(str(tmp_path), "missing.bin"), f)


@pytest.mark.parametrize("layout", [(63, 24, 0, 0, 8, 8), (64, 24, 30, 0, 3, 3),
                                    (64, 24, 0, 20, 8, 5), (64, 24, 0, 0, 0, 4)])
def test_layout_validation(cpi, tmp_path, layout):
    path = os.path.join(str(tmp_path), "x.bin")
    open(path, "wb").close()
    with pytest.raises(cpi.CpiError) as e:
        cpi.file_frames(path, cpi.SideBySide(*layout))
    assert e.value.status == 1
