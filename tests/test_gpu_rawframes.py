"""Raw side-by-side sensor frames on the device: the split into the two
detectors' regions of interest, and file streaming into the running sums,
against the oracle's correlation of the same detector frames (bit-exact)."""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, compose_sidebyside, generate_frames, pack_bits_lsb, \
    pack_raw_frames, write_frame_files
from tests.gpu_util import assert_bit_exact, dev, log, oracle_in_layout, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


@pytest.mark.parametrize("layout", [(64, 20, 3, 2, 13, 5), (64, 24, 0, 0, 32, 24),
                                    (512, 8, 8, 1, 240, 7), (18, 3, 1, 0, 7, 3)])
def test_split_matches_slicing(cpi, layout):
    import torch

    fw, fh, rx, ry, rw, rh = layout
    n = 37
    rng = np.random.default_rng(fw * 100 + rw)
    raw = (rng.random((n, fh, fw)) < 0.4).astype(np.uint8)
    packed = pack_raw_frames(raw)
    half = fw // 2
    want_a = pack_bits_lsb(raw[:, ry:ry + rh, rx:rx + rw].reshape(n, -1))
    want_b = pack_bits_lsb(raw[:, ry:ry + rh, half + rx:half + rx + rw].reshape(n, -1))
    f = cpi.SideBySide(*layout)
    log(f"case split layout={layout}")
    d_in = to_dev(np.concatenate([packed.reshape(-1), np.zeros(16, np.uint8)]))
    ob = (rw * rh + 7) // 8
    out_a = torch.full((n * ob,), 0xAB, dtype=torch.uint8, device=dev())
    out_b = torch.full((n * ob,), 0xAB, dtype=torch.uint8, device=dev())
    cpi.split_sidebyside(d_in, n, f, out_a, out_b)
    torch.cuda.synchronize()
    assert np.array_equal(out_a.cpu().numpy().reshape(n, ob), want_a)
    assert np.array_equal(out_b.cpu().numpy().reshape(n, ob), want_b)


def _ingest(cpi, paths, f, max_chunk, host_frames, dev_frames):
    import torch

    st = cpi.Stream(f.roi_pixels, f.roi_pixels, cpi.FRAMES_BIT1, max_chunk=max_chunk,
                    device=dev())
    ha = torch.empty(host_frames * f.frame_bytes, dtype=torch.uint8).pin_memory()
    hb = torch.empty(host_frames * f.frame_bytes, dtype=torch.uint8).pin_memory()
    raw = torch.empty(dev_frames * f.frame_bytes, dtype=torch.uint8, device=dev())
    k = st.ingest_files(paths, f, ha, hb, raw)
    torch.cuda.synchronize()
    return st, k


@pytest.mark.parametrize("pieces", [(50, 30, 64), (40, 40, 7), (1000, 1000, 1000)])
def test_ingest_files_matches_oracle(cpi, tmp_path, pieces):
    """Three files of 100, 37 and 64 frames, read in pieces bounded by the
    stream's chunk and both buffers, give the oracle's Gamma bit for bit."""
    import torch

    max_chunk, host_frames, dev_frames = pieces
    rng = np.random.default_rng(11)
    n, rh, rw = 201, 12, 16
    a = (rng.random((n, rh, rw)) < 0.15).astype(np.uint8)
    b = (rng.random((n, rh, rw)) < 0.25).astype(np.uint8)
    raw = compose_sidebyside(a, b, frame_w=64, frame_h=24, roi_x=5, roi_y=3, rng=rng)
    paths = write_frame_files(str(tmp_path), pack_raw_frames(raw), [100, 37, 64])
    f = cpi.sidebyside(64, 24, 5, 3, rw, rh)
    log(f"case ingest files pieces={pieces}")
    st, k = _ingest(cpi, paths, f, max_chunk, host_frames, dev_frames)
    assert k == n and st.frames == n
    p = rw * rh
    out = {"gamma": torch.empty(p * p, dtype=torch.float64, device=dev()),
           "gamma_f32": torch.empty(p * p, dtype=torch.float32, device=dev()),
           "numer": torch.empty(p * p, dtype=torch.int64, device=dev()),
           "sum_a": torch.empty(p, dtype=torch.int64, device=dev()),
           "sum_b": torch.empty(p, dtype=torch.int64, device=dev())}
    st.gamma(cpi.GAMMA_VIEW_MAJOR, **out)
    torch.cuda.synchronize()
    got = {key: v.cpu().numpy() for key, v in out.items()}
    ref = oracle.correlation(a.reshape(n, -1), b.reshape(n, -1), n, p, p, oracle.FRAMES_U8)
    assert_bit_exact(got, oracle_in_layout(ref, cpi.GAMMA_VIEW_MAJOR))
    st.close()


def test_ingest_paper_file_layout(cpi, tmp_path):
    """The paper's file layout (256 x 512 frames, 512 per file) with a 32 x 32
    region of interest of the streaming workload's frames, two files."""
    import torch

    w = WORKLOADS["da128_db64_stream200x1000_bit1"]
    a8, b8 = generate_frames(w, count=1024)
    # take a 32 x 32 region of detector A, and the upsampled 16 x 16 centre of B
    a = a8.reshape(-1, w.ha, w.wa)[:, 40:72, 40:72]
    b = np.repeat(np.repeat(b8.reshape(-1, w.hb, w.wb)[:, 24:40, 24:40], 2, axis=1), 2, axis=2)
    rng = np.random.default_rng(5)
    raw = compose_sidebyside(a, b, frame_w=512, frame_h=256, roi_x=100, roi_y=60, rng=rng)
    paths = write_frame_files(str(tmp_path), pack_raw_frames(raw), 512)
    f = cpi.sidebyside(512, 256, 100, 60, 32, 32)
    assert [cpi.file_frames(p_, f) for p_ in paths] == [512, 512]
    log("case ingest paper file layout")
    st, k = _ingest(cpi, paths, f, 512, 256, 256)
    assert k == 1024
    p = 32 * 32
    g = torch.empty(p * p, dtype=torch.float64, device=dev())
    st.gamma(cpi.GAMMA_VIEW_MAJOR, gamma=g)
    torch.cuda.synchronize()
    ref = oracle.correlation(a.reshape(1024, -1), b.reshape(1024, -1), 1024, p, p,
                             oracle.FRAMES_U8)
    assert np.array_equal(g.cpu().numpy(), oracle.to_layout(ref["gamma"], oracle.GAMMA_VIEW_MAJOR).reshape(-1))
    st.close()


def test_ingest_rejects_mismatched_stream(cpi, tmp_path):
    import torch

    raw = np.zeros((4, 8, 32), np.uint8)
    paths = write_frame_files(str(tmp_path), pack_raw_frames(raw), 4)
    f = cpi.sidebyside(32, 8, 0, 0, 8, 8)
    st = cpi.Stream(60, 64, cpi.FRAMES_BIT1, max_chunk=8, device=dev())
    ha = torch.empty(8 * f.frame_bytes, dtype=torch.uint8)
    hb = torch.empty(8 * f.frame_bytes, dtype=torch.uint8)
    raw_d = torch.empty(8 * f.frame_bytes, dtype=torch.uint8, device=dev())
    with pytest.raises(cpi.CpiError) as e:
        st.ingest_files(paths, f, ha, hb, raw_d)
    assert e.value.status == 1
    st.close()
