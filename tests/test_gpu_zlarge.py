"""Full-size checks on the large workload: Da 256x256, Db 128x128, N = 100000
1-bit frames, 128 refocus planes (the configuration whose Gamma is
65536 x 16384).  Frames are generated on the device (seeded).

Gamma (8.6 GB in FP64) cannot go through the CPU oracle whole, so it is
checked (a) element by element against the oracle on sampled pixel pairs,
computed from those pixels' frame columns only, (b) through integer
identities over every entry: row sums, column sums and Freivalds products of
the exact numerator, recovered as rint(Gamma * N^2) (|numer| < 2^52 here).
Refocusing is checked at full size through the alpha = 1 plane, which equals
the row sums of Gamma over the views (an identity tied to the frames), against
the FP64 oracle on 25 planes of the 128-plane stack (sampled pixels plus each
plane's largest-magnitude pixel, on the device Gamma that the identities above
tie to the frames), and through a closed-form point phantom at the full
geometry.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, alphas_for
from synth.gpu_speckle import generate_binary_frames_gpu
from tests.gpu_util import dev, log, plane_rel_err

pytestmark = pytest.mark.gpu

W = WORKLOADS["da256_db128_n100000_bit1"]


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


@pytest.fixture(scope="module")
def large(cpi):
    import torch

    log(f"case {W.name}: generating frames on the device")
    fa, fb = generate_binary_frames_gpu(W, device=dev())
    n, pa, pb = W.n_frames, W.pa, W.pb
    gamma = torch.empty(pa * pb, dtype=torch.float64, device=dev())
    g32 = torch.empty(pa * pb, dtype=torch.float32, device=dev())
    sa = torch.empty(pa, dtype=torch.int64, device=dev())
    sb = torch.empty(pb, dtype=torch.int64, device=dev())
    log("case large: correlate")
    cpi.correlate(fa.reshape(-1), fb.reshape(-1), n, pa, pb, cpi.FRAMES_BIT1,
                  cpi.GAMMA_VIEW_MAJOR, gamma=gamma, gamma_f32=g32, sum_a=sa, sum_b=sb)
    torch.cuda.synchronize()
    return fa, fb, gamma, g32, sa, sb


def _columns(packed, pix):
    """0/1 values of the listed pixels in every frame, from packed bytes (host)."""
    pix = np.asarray(pix)
    return ((packed[:, pix // 8] >> (pix % 8)) & 1).astype(np.uint8)


def _unpacked_chunks(torch, packed, npix, step=10000):
    bits = torch.arange(8, device=packed.device, dtype=torch.uint8)
    for lo in range(0, packed.shape[0], step):
        c = packed[lo:lo + step]
        u = ((c.unsqueeze(2) >> bits) & 1).reshape(c.shape[0], -1)[:, :npix]
        yield lo, u


def test_sampled_entries_match_oracle(cpi, large):
    fa, fb, gamma, g32, sa, sb = large
    n, pa, pb = W.n_frames, W.pa, W.pb
    rng = np.random.default_rng(31)
    rows = np.sort(rng.choice(pa, 512, replace=False))
    views = np.sort(rng.choice(pb, 24, replace=False))
    ha = fa.cpu().numpy()
    hb = fb.cpu().numpy()
    a = _columns(ha, rows)
    b = _columns(hb, views)
    log("case large: oracle on sampled pairs")
    ref = oracle.correlation(a, b, n, rows.size, views.size, oracle.FRAMES_U8)
    g = gamma.view(pb, pa)[views][:, rows].cpu().numpy()
    assert np.array_equal(g, ref["gamma"].T)
    assert np.array_equal(g32.view(pb, pa)[views][:, rows].cpu().numpy(), ref["gamma_f32"].T)
    assert np.array_equal(sa.cpu().numpy()[rows], ref["sum_a"])
    assert np.array_equal(sb.cpu().numpy()[views], ref["sum_b"])


def test_integer_identities_over_every_entry(cpi, large):
    import torch

    fa, fb, gamma, g32, sa, sb = large
    n, pa, pb = W.n_frames, W.pa, W.pb
    d = dev()
    num = torch.round(gamma.view(pb, pa) * float(n * n))            # exact integers in FP64
    # rows of A (sum over views) and of B (sum over A pixels), from the frames
    tb = torch.zeros(n, dtype=torch.float64, device=d)               # |B_i|
    ta = torch.zeros(n, dtype=torch.float64, device=d)               # |A_i|
    for lo, u in _unpacked_chunks(torch, fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    for lo, u in _unpacked_chunks(torch, fa, pa):
        ta[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    rng = np.random.default_rng(32)
    v = torch.from_numpy(rng.integers(-2, 3, size=pa).astype(np.float64)).to(d)
    a_tb = torch.zeros(pa, dtype=torch.float64, device=d)            # sum_i A_i[p] |B_i|
    a_v = torch.zeros(n, dtype=torch.float64, device=d)              # A v
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
    assert torch.equal(sa_f, sa.to(torch.float64)) and torch.equal(sb_f, sb.to(torch.float64))
    log("case large: row/column sums and Freivalds")
    rows_a = n * a_tb - sa_f * sb_f.sum()
    rows_b = n * b_ta - sb_f * sa_f.sum()
    assert torch.equal(num.sum(dim=0), rows_a)
    assert torch.equal(num.sum(dim=1), rows_b)
    assert torch.equal(num @ v, n * bt_av - sb_f * (sa_f @ v))
    # FP32 copy is the rounding of FP64
    assert torch.equal(g32, gamma.to(torch.float32))


def _stack_alphas():
    al = list(alphas_for(W))
    al[len(al) // 2] = 1.0
    return al


@pytest.fixture(scope="module")
def stack(cpi, large):
    """The 128-plane stack of the workload (its alpha grid with the middle
    plane set to alpha = 1), refocused in one batched call."""
    import torch

    fa, fb, gamma, g32, sa, sb = large
    geo = cpi.geometry_default(W.wa, W.ha, W.wb, W.hb)
    al = _stack_alphas()
    out = torch.empty(len(al) * W.pa, dtype=torch.float32, device=dev())
    log("case large: refocus 128 planes")
    cpi.refocus(g32, geo, al, out)
    torch.cuda.synchronize()
    return al, out


def test_refocus_alpha_one_is_row_sum(cpi, large, stack):
    import torch

    fa, fb, gamma, g32, sa, sb = large
    n, pa, pb = W.n_frames, W.pa, W.pb
    al, out = stack
    # alpha = 1 plane against the frames' row sums / N^2 (no Gamma in between)
    tb = torch.zeros(n, dtype=torch.float64, device=dev())
    for lo, u in _unpacked_chunks(torch, fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    a_tb = torch.zeros(pa, dtype=torch.float64, device=dev())
    for lo, u in _unpacked_chunks(torch, fa, pa):
        a_tb += u.to(torch.float64).t() @ tb[lo:lo + u.shape[0]]
    rows = (n * a_tb - sa.to(torch.float64) * float(sb.sum())) / float(n * n)
    got = out.view(len(al), pa)[len(al) // 2].to(torch.float64)
    err = plane_rel_err(got.cpu().numpy()[None], rows.cpu().numpy()[None])
    log(f"alpha=1 plane relative error {err.max():.3g}")
    assert err.max() <= 1e-5
    assert torch.isfinite(out).all()


def test_refocus_point_phantom_full_geometry(cpi):
    """Closed-form point Gamma at Da 256x256, Db 128x128: the refocused plane
    at alpha* peaks exactly at the point with the closed-form value."""
    import torch

    g = oracle.default_geometry(W.wa, W.ha, W.wb, W.hb)
    alpha_star, xo, yo = 0.8, 101, 147
    d = dev()
    xb = torch.arange(g.wb, device=d, dtype=torch.float64)
    yb = torch.arange(g.hb, device=d, dtype=torch.float64)
    px = alpha_star * (xo - g.ca_x) + g.ca_x + (1 - alpha_star) * g.mag_x * (xb - g.cb_x)
    py = alpha_star * (yo - g.ca_y) + g.ca_y + (1 - alpha_star) * g.mag_y * (yb - g.cb_y)
    x0, y0 = torch.floor(px), torch.floor(py)
    fx, fy = px - x0, py - y0
    gam = torch.zeros(g.hb, g.wb, g.ha, g.wa, dtype=torch.float32, device=d)
    iy, ix = torch.meshgrid(torch.arange(g.hb, device=d), torch.arange(g.wb, device=d), indexing="ij")
    for dy in (0, 1):
        for dx in (0, 1):
            wy = fy if dy else 1 - fy
            wx = fx if dx else 1 - fx
            gam[iy, ix, (y0.long() + dy)[iy], (x0.long() + dx)[ix]] = (wy[iy] * wx[ix]).to(torch.float32)
    peak = float((((1 - fx) ** 2 + fx ** 2).sum() * ((1 - fy) ** 2 + fy ** 2).sum()))
    out = torch.empty(g.ha * g.wa, dtype=torch.float32, device=d)
    log("case large: point phantom")
    cpi.refocus(gam.reshape(-1), cpi.make_geometry(**g.__dict__), [alpha_star], out)
    torch.cuda.synchronize()
    img = out.view(g.ha, g.wa)
    assert abs(float(img[yo, xo]) - peak) <= 1e-5 * peak
    assert int(torch.argmax(img)) == yo * g.wa + xo


def test_refocus_stack_planes_vs_oracle(cpi, large, stack):
    """25 planes of the 128-plane stack (24 evenly spaced, first and last
    included, plus the alpha = 1 plane) against the FP64 oracle at 64 sampled
    pixels plus each checked plane's largest-magnitude pixel.  The oracle
    refocuses the device Gamma64, which the tests above show to be the exact
    Gamma of the frames; per plane, max error / max magnitude <= 1e-5."""
    fa, fb, gamma, g32, sa, sb = large
    al, out = stack
    na = len(al)
    planes = np.unique(np.concatenate([np.linspace(0, na - 1, 24).round().astype(int),
                                       [na // 2]]))
    got = out.view(na, W.ha, W.wa)[planes].cpu().numpy()
    rng = np.random.default_rng(33)
    ys = list(rng.integers(0, W.ha, 64))
    xs = list(rng.integers(0, W.wa, 64))
    flat = np.abs(got.reshape(planes.size, -1))
    for k in range(planes.size):
        yy, xx = np.unravel_index(np.argmax(flat[k]), (W.ha, W.wa))
        ys.append(yy)
        xs.append(xx)
    ys, xs = np.array(ys), np.array(xs)
    g = oracle.default_geometry(W.wa, W.ha, W.wb, W.hb)
    log(f"case large: oracle refocus of {planes.size} planes at {ys.size} pixels")
    want = oracle.refocus_pixels(gamma.cpu().numpy(), g, np.asarray(al)[planes], ys, xs)
    err = plane_rel_err(got[:, ys, xs], want)
    for k, e in zip(planes, err):
        log(f"plane {k} alpha {al[k]:.6f}: relative error {e:.3g}")
    assert err.max() <= 1e-5
