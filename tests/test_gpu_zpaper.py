"""The paper's benchmark configuration: 256 x 256 regions on both detectors
(Gamma 65536 x 65536), 11 files of 512 1-bit frames, 261 refocus planes.
Frames are generated on the device (seeded).

Gamma (34 GB in FP64) is checked element by element against the oracle on
sampled pixel pairs, computed from those pixels' frame columns only, and
through integer identities over every entry: row sums, column sums and
Freivalds products of the exact numerator, recovered as rint(Gamma * N^2)
(|numer| < 2^52 here).  The 261-plane refocus is checked at full size through
the alpha = 1 plane, which equals the row sums of Gamma over the views (an
identity tied to the frames), and against the FP64 oracle on 25 of its planes
(sampled pixels plus each plane's largest-magnitude pixel, on the device Gamma
that the identities tie to the frames; three groups of planes, one test each).
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, alphas_for
from synth.gpu_speckle import generate_binary_frames_gpu
from tests.gpu_util import dev, log, plane_rel_err

pytestmark = pytest.mark.gpu

W = WORKLOADS["da256_db256_files11_bit1"]


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


@pytest.fixture(scope="module")
def paper(cpi):
    import torch

    log(f"case {W.name}: generating frames on the device")
    fa, fb = generate_binary_frames_gpu(W, device=dev())
    n, pa, pb = W.n_frames, W.pa, W.pb
    gamma = torch.empty(pa * pb, dtype=torch.float64, device=dev())
    g32 = torch.empty(pa * pb, dtype=torch.float32, device=dev())
    sa = torch.empty(pa, dtype=torch.int64, device=dev())
    sb = torch.empty(pb, dtype=torch.int64, device=dev())
    log("case paper: correlate")
    cpi.correlate(fa.reshape(-1), fb.reshape(-1), n, pa, pb, cpi.FRAMES_BIT1,
                  cpi.GAMMA_VIEW_MAJOR, gamma=gamma, gamma_f32=g32, sum_a=sa, sum_b=sb)
    torch.cuda.synchronize()
    return fa, fb, gamma, g32, sa, sb


def _columns(packed, pix):
    pix = np.asarray(pix)
    return ((packed[:, pix // 8] >> (pix % 8)) & 1).astype(np.uint8)


def _unpacked_chunks(torch, packed, npix, step=2816):
    bits = torch.arange(8, device=packed.device, dtype=torch.uint8)
    for lo in range(0, packed.shape[0], step):
        c = packed[lo:lo + step]
        u = ((c.unsqueeze(2) >> bits) & 1).reshape(c.shape[0], -1)[:, :npix]
        yield lo, u


def test_sampled_entries_match_oracle(cpi, paper):
    fa, fb, gamma, g32, sa, sb = paper
    n, pa, pb = W.n_frames, W.pa, W.pb
    rng = np.random.default_rng(41)
    rows = np.sort(rng.choice(pa, 384, replace=False))
    views = np.sort(rng.choice(pb, 32, replace=False))
    a = _columns(fa.cpu().numpy(), rows)
    b = _columns(fb.cpu().numpy(), views)
    log("case paper: oracle on sampled pairs")
    ref = oracle.correlation(a, b, n, rows.size, views.size, oracle.FRAMES_U8)
    assert np.array_equal(gamma.view(pb, pa)[views][:, rows].cpu().numpy(), ref["gamma"].T)
    assert np.array_equal(g32.view(pb, pa)[views][:, rows].cpu().numpy(), ref["gamma_f32"].T)
    assert np.array_equal(sa.cpu().numpy()[rows], ref["sum_a"])
    assert np.array_equal(sb.cpu().numpy()[views], ref["sum_b"])


def test_integer_identities_over_every_entry(cpi, paper):
    import torch

    fa, fb, gamma, g32, sa, sb = paper
    n, pa, pb = W.n_frames, W.pa, W.pb
    d = dev()
    num = torch.round(gamma.view(pb, pa) * float(n * n))
    ta = torch.zeros(n, dtype=torch.float64, device=d)
    tb = torch.zeros(n, dtype=torch.float64, device=d)
    for lo, u in _unpacked_chunks(torch, fa, pa):
        ta[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    for lo, u in _unpacked_chunks(torch, fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    rng = np.random.default_rng(42)
    v = torch.from_numpy(rng.integers(-2, 3, size=pa).astype(np.float64)).to(d)
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
    assert torch.equal(sa_f, sa.to(torch.float64)) and torch.equal(sb_f, sb.to(torch.float64))
    log("case paper: row/column sums and Freivalds")
    assert torch.equal(num.sum(dim=0), n * a_tb - sa_f * sb_f.sum())
    assert torch.equal(num.sum(dim=1), n * b_ta - sb_f * sa_f.sum())
    assert torch.equal(num @ v, n * bt_av - sb_f * (sa_f @ v))
    assert torch.equal(g32, gamma.to(torch.float32))


@pytest.fixture(scope="module")
def stack(cpi, paper):
    """The 261-plane stack, refocused in one batched call."""
    import torch

    fa, fb, gamma, g32, sa, sb = paper
    geo = cpi.geometry_default(W.wa, W.ha, W.wb, W.hb)
    al = list(alphas_for(W))
    assert al[130] == 1.0          # linspace(0.5, 1.5, 261) holds alpha = 1 exactly
    out = torch.empty(len(al) * W.pa, dtype=torch.float32, device=dev())
    log("case paper: refocus 261 planes")
    cpi.refocus(g32, geo, al, out)
    torch.cuda.synchronize()
    return al, out


@pytest.fixture(scope="module")
def gamma_host(paper):
    """The device Gamma64 on the host, once for the oracle's checks."""
    log("case paper: Gamma to the host")
    return paper[2].cpu().numpy()


def test_refocus_261_planes_alpha_one(cpi, paper, stack):
    import torch

    fa, fb, gamma, g32, sa, sb = paper
    n, pa, pb = W.n_frames, W.pa, W.pb
    al, out = stack
    assert torch.isfinite(out).all()
    tb = torch.zeros(n, dtype=torch.float64, device=dev())
    for lo, u in _unpacked_chunks(torch, fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    a_tb = torch.zeros(pa, dtype=torch.float64, device=dev())
    for lo, u in _unpacked_chunks(torch, fa, pa):
        a_tb += u.to(torch.float64).t() @ tb[lo:lo + u.shape[0]]
    rows = (n * a_tb - sa.to(torch.float64) * float(sb.sum())) / float(n * n)
    got = out.view(len(al), pa)[130].to(torch.float64)
    err = plane_rel_err(got.cpu().numpy()[None], rows.cpu().numpy()[None])
    log(f"alpha=1 plane relative error {err.max():.3g}")
    assert err.max() <= 1e-5


# 24 evenly spaced planes of the 261 (first and last included) plus alpha = 1,
# in three groups so that each oracle run stays short
_PLANES = np.unique(np.concatenate([np.linspace(0, 260, 24).round().astype(int), [130]]))
_GROUPS = [_PLANES[0::3], _PLANES[1::3], _PLANES[2::3]]


@pytest.mark.parametrize("group", range(len(_GROUPS)))
def test_refocus_planes_vs_oracle(cpi, stack, gamma_host, group):
    """Planes of the 261-plane stack against the FP64 oracle at 48 sampled
    pixels plus each checked plane's largest-magnitude pixel; per plane, max
    error / max magnitude <= 1e-5."""
    al, out = stack
    planes = _GROUPS[group]
    got = out.view(len(al), W.ha, W.wa)[planes].cpu().numpy()
    rng = np.random.default_rng(43 + group)
    ys = list(rng.integers(0, W.ha, 48))
    xs = list(rng.integers(0, W.wa, 48))
    flat = np.abs(got.reshape(planes.size, -1))
    for k in range(planes.size):
        yy, xx = np.unravel_index(np.argmax(flat[k]), (W.ha, W.wa))
        ys.append(yy)
        xs.append(xx)
    ys, xs = np.array(ys), np.array(xs)
    g = oracle.default_geometry(W.wa, W.ha, W.wb, W.hb)
    log(f"case paper: oracle refocus of planes {list(planes)} at {ys.size} pixels")
    want = oracle.refocus_pixels(gamma_host, g, np.asarray(al)[planes], ys, xs)
    err = plane_rel_err(got[:, ys, xs], want)
    for k, e in zip(planes, err):
        log(f"plane {k} alpha {al[k]:.6f}: relative error {e:.3g}")
    assert err.max() <= 1e-5
