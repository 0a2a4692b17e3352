"""Memory-adaptive blocking at the paper's pixel counts: 256 x 256 regions on
both detectors (Gamma 65536 x 65536) and the paper's full frame count,
3997696 distinct 1-bit frames (7808 files of 512), made on the device
(seeded).  The workspace given to cpi_correlate holds the running sums and
about 480000 frames' operands, not the one-shot operands of all frames, so the
frames are folded in several blocks.

Gamma is checked against the oracle on sampled pixel pairs (from those
pixels' frame columns only) and through integer identities over every entry:
row sums, column sums and a Freivalds product of the exact numerator,
recovered as rint(Gamma * N^2) (exact: |numer| <= N^2 / 4 < 2^52, so the two
roundings move Gamma * N^2 by at most |numer| * 2^-52 < 0.01), evaluated in int64, and the FP32 Gamma is the rounding of the FP64 one."""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS
from synth.gpu_speckle import generate_binary_frames_gpu
from tests.gpu_util import dev, log

pytestmark = pytest.mark.gpu

W = WORKLOADS["da256_db256_files11_bit1"]
N = 7808 * 512


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def _columns(torch, packed, pix):
    """0/1 values of the listed pixels in every frame (gathered on the device)."""
    pix = torch.from_numpy(np.asarray(pix)).to(packed.device)
    return ((packed[:, pix // 8] >> (pix % 8).to(torch.uint8)) & 1).cpu().numpy()


def _unpacked_chunks(torch, packed, npix, step=8192):
    bits = torch.arange(8, device=packed.device, dtype=torch.uint8)
    for lo in range(0, packed.shape[0], step):
        c = packed[lo:lo + step]
        yield lo, ((c.unsqueeze(2) >> bits) & 1).reshape(c.shape[0], -1)[:, :npix]


def test_blocked_correlate_paper_pixels_paper_frames(cpi):
    import torch

    n, pa, pb = N, W.pa, W.pb
    d = dev()
    log(f"case paper pixels, {n} frames: generating on the device")
    fa, fb = generate_binary_frames_gpu(W, count=n, device=d)
    full = cpi.correlate_workspace_size(n, pa, pb, cpi.FRAMES_BIT1)
    limit = 25 << 30
    assert limit < full
    gamma = torch.empty(pa * pb, dtype=torch.float64, device=d)
    g32 = torch.empty(pa * pb, dtype=torch.float32, device=d)
    sa = torch.empty(pa, dtype=torch.int64, device=d)
    sb = torch.empty(pb, dtype=torch.int64, device=d)
    log(f"case paper pixels: blocked correlate, workspace {limit} of {full} bytes")
    ws = cpi.alloc_workspace(limit, d)
    cpi.correlate(fa.reshape(-1), fb.reshape(-1), n, pa, pb, cpi.FRAMES_BIT1,
                  cpi.GAMMA_VIEW_MAJOR, gamma=gamma, gamma_f32=g32, sum_a=sa, sum_b=sb,
                  workspace=ws)
    torch.cuda.synchronize()
    del ws
    torch.cuda.empty_cache()
    assert torch.equal(g32, gamma.to(torch.float32))

    # sampled pairs against the oracle
    rng = np.random.default_rng(43)
    rows = np.sort(rng.choice(pa, 256, replace=False))
    views = np.sort(rng.choice(pb, 16, replace=False))
    log("case paper pixels: oracle on sampled pairs")
    a = _columns(torch, fa, rows)
    b = _columns(torch, fb, views)
    ref = oracle.correlation(a, b, n, rows.size, views.size, oracle.FRAMES_U8)
    del a, b
    assert np.array_equal(gamma.view(pb, pa)[views][:, rows].cpu().numpy(), ref["gamma"].T)
    assert np.array_equal(sa.cpu().numpy()[rows], ref["sum_a"])
    assert np.array_equal(sb.cpu().numpy()[views], ref["sum_b"])

    # identities over every entry, from the frames: the frame-side products
    # are integers below 2^53 (exact in FP64), the identities are evaluated
    # in int64 (their terms reach 2^59)
    log("case paper pixels: row/column sums and Freivalds")
    num = torch.round(gamma.view(pb, pa) * float(n * n)).to(torch.int64)
    del gamma
    torch.cuda.empty_cache()
    ta = torch.zeros(n, dtype=torch.float64, device=d)
    tb = torch.zeros(n, dtype=torch.float64, device=d)
    for lo, u in _unpacked_chunks(torch, fa, pa):
        ta[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    for lo, u in _unpacked_chunks(torch, fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    vi = rng.integers(-2, 3, size=pa)
    v = torch.from_numpy(vi.astype(np.float64)).to(d)
    a_tb = torch.zeros(pa, dtype=torch.float64, device=d)
    a_v = torch.zeros(n, dtype=torch.float64, device=d)
    sa_f = torch.zeros(pa, dtype=torch.float64, device=d)
    for lo, u in _unpacked_chunks(torch, fa, pa):
        uf = u.to(torch.float64)
        a_tb += uf.t() @ tb[lo:lo + u.shape[0]]
        a_v[lo:lo + u.shape[0]] = uf @ v
        sa_f += uf.sum(dim=0)
    b_ta = torch.zeros(pb, dtype=torch.float64, device=d)
    bt_av = torch.zeros(pb, dtype=torch.float64, device=d)
    sb_f = torch.zeros(pb, dtype=torch.float64, device=d)
    for lo, u in _unpacked_chunks(torch, fb, pb):
        uf = u.to(torch.float64)
        b_ta += uf.t() @ ta[lo:lo + u.shape[0]]
        bt_av += uf.t() @ a_v[lo:lo + u.shape[0]]
        sb_f += uf.sum(dim=0)
    i64 = torch.int64
    sa_i, sb_i = sa_f.to(i64), sb_f.to(i64)
    assert torch.equal(sa_i, sa) and torch.equal(sb_i, sb)
    assert torch.equal(num.sum(dim=0), n * a_tb.to(i64) - sa_i * sb_i.sum())
    assert torch.equal(num.sum(dim=1), n * b_ta.to(i64) - sb_i * sa_i.sum())
    vd = torch.from_numpy(vi.astype(np.int64)).to(d)
    nv = torch.cat([(num[r:r + 2048] * vd).sum(dim=1) for r in range(0, pb, 2048)])
    assert torch.equal(nv, n * bt_av.to(i64) - sb_i * (sa_i * vd).sum())
