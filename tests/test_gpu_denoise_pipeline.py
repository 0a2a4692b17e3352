"""GPU checks of the denoiser's place in the pipeline: training pairs are the
planes of one stream after a prefix of its frames (checked against the FP64
oracle's refocus of the oracle's Gamma of that prefix, 1e-5 relative per
plane), and the fallback to the plain planes."""
import numpy as np
import pytest

import oracle
from synth import Workload, generate_frames, pack_bits_lsb
from tests.gpu_util import dev, log, plane_rel_err

pytestmark = pytest.mark.gpu

W = Workload("tiny_denoise", 9, 16, 16, 8, 8, 300, "binary_packed", 4)


@pytest.fixture(scope="module")
def mods():
    import paper_2407_20692_amd as cpi
    import paper_2407_20692_amd.denoise_pipeline as dp
    import paper_2407_20692_amd.denoiser as dn
    return cpi, dp, dn


def test_prefix_planes_match_oracle(mods):
    import torch
    cpi, dp, _ = mods
    ua, ub = generate_frames(W)
    fa, fb = pack_bits_lsb(ua), pack_bits_lsb(ub)
    alphas = np.array([0.6, 0.9, 1.0, 1.4])
    geo = cpi.geometry_default(W.wa, W.ha, W.wb, W.hb)
    g = oracle.default_geometry(W.wa, W.ha, W.wb, W.hb)
    counts = [50, 172, 300]     # frame slices stay 16-byte aligned (8-byte B frames)
    outs = [torch.full((4, 16, 16), np.nan, dtype=torch.float32, device=dev()) for _ in counts]
    dp.prefix_planes(torch.from_numpy(fa).to(dev()), torch.from_numpy(fb).to(dev()), W.pa, W.pb,
                     geo, alphas, counts, outs, chunk=64)
    torch.cuda.synchronize()
    for n, out in zip(counts, outs):
        r = oracle.correlation(fa[:n], fb[:n], n, W.pa, W.pb, oracle.FRAMES_BIT1)
        gam = oracle.to_layout(r["gamma"], oracle.GAMMA_VIEW_MAJOR)
        ref = oracle.refocus(gam, g, alphas)
        err = plane_rel_err(out.cpu().numpy(), ref)
        log(f"prefix {n}: max plane rel err {max(err):.2e}")
        assert max(err) <= 1e-5


def test_fallback_rules(mods):
    import torch
    _, dp, dn = mods
    rng = np.random.default_rng(3)
    few = torch.from_numpy(rng.standard_normal((3, 16, 16)).astype(np.float32)).to(dev())
    plain = torch.from_numpy(rng.standard_normal((3, 16, 16)).astype(np.float32)).to(dev())
    net = dn.Denoiser(seed=2, device=dev())
    off = dp.decide(20.0, 0.5, 21.0, 0.6, 500, 4000)
    assert not off.use_denoiser
    assert dp.apply(net, off, few, plain) is plain
    assert dp.apply(None, None, few) is few
    on = dp.decide(22.0, 0.7, 21.0, 0.6, 500, 4000)
    assert on.use_denoiser
    out = dp.apply(net, on, few)
    assert torch.isfinite(out).all()
    ref = net.forward(few)
    assert torch.equal(out, ref)
    # a network whose output is not finite falls back to the plain input
    net.params.fill_(float("nan"))
    out = dp.apply(net, on, few)
    assert torch.equal(out, few)
