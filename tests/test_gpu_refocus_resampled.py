"""GPU parity of refocusing with a resampled lens-plane grid (the general
4-D multilinear interpolation) against the FP64 oracle: per plane,
max |I_gpu - I_oracle| / max |I_oracle| <= 1e-5 (the refocus tolerance),
with the oracle evaluating all 16 corners of every sample directly."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, log, plane_rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def _run(cpi, gam32, g, s, alphas):
    import torch
    geo = cpi.make_geometry(**g.__dict__)
    ls = cpi.lens_sampling(s.nx, s.ny, s.ox, s.oy, s.sx, s.sy)
    out = torch.full((len(alphas) * g.out_h * g.out_w,), np.nan, dtype=torch.float32, device=dev())
    cpi.refocus_resampled(to_dev(gam32), geo, ls, alphas, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(alphas), g.out_h, g.out_w)


SMALL = [
    ("half_step", oracle.LensSampling(15, 15, 0.0, 0.0, 0.5, 0.5)),
    ("irregular", oracle.LensSampling(7, 5, -0.3, 0.4, 1.15, 1.6)),
    ("coarse_outside", oracle.LensSampling(3, 4, -1.5, -0.75, 3.5, 2.75)),
    ("single", oracle.LensSampling(1, 1, 3.25, 4.5, 1.0, 1.0)),
]


@pytest.mark.parametrize("name,s", SMALL, ids=[n for n, _ in SMALL])
def test_resampled_matches_oracle(cpi, name, s):
    g = oracle.default_geometry(16, 16, 8, 8)
    rng = np.random.default_rng(abs(hash(name)) % 2**32)
    gam32 = rng.standard_normal(g.wa * g.ha * g.wb * g.hb).astype(np.float32)
    alphas = np.linspace(0.5, 1.5, 5)
    got = _run(cpi, gam32, g, s, alphas)
    ref = oracle.refocus_resampled(gam32.astype(np.float64), g, s, alphas)
    err = plane_rel_err(got, ref)
    log(f"resampled {name}: max plane rel err {err.max():.2e}")
    assert err.max() <= TOL


def test_integer_grid_equals_refocus(cpi):
    import torch
    g = oracle.default_geometry(20, 12, 10, 6)
    rng = np.random.default_rng(5)
    gam32 = rng.standard_normal(g.wa * g.ha * g.wb * g.hb).astype(np.float32)
    alphas = np.array([0.6, 1.0, 1.3])
    s = oracle.LensSampling(g.wb, g.hb, 0.0, 0.0, 1.0, 1.0)
    got = _run(cpi, gam32, g, s, alphas)
    out = torch.empty(len(alphas) * g.out_h * g.out_w, dtype=torch.float32, device=dev())
    cpi.refocus(to_dev(gam32), cpi.make_geometry(**g.__dict__), alphas, out)
    torch.cuda.synchronize()
    assert np.array_equal(got, out.cpu().numpy().reshape(got.shape))


def test_resample_views_entry_point(cpi):
    """The views step on its own: each resampled view is the bilinear mix of
    its four neighbours (checked against the oracle at alpha = 1, where the
    refocused plane is the plain sum of the views)."""
    import torch
    g = oracle.default_geometry(8, 8, 4, 4)
    rng = np.random.default_rng(6)
    gam32 = rng.standard_normal(g.wa * g.ha * g.wb * g.hb).astype(np.float32)
    s = oracle.LensSampling(5, 3, 0.25, -0.5, 0.7, 1.5)
    ls = cpi.lens_sampling(s.nx, s.ny, s.ox, s.oy, s.sx, s.sy)
    geo = cpi.make_geometry(**g.__dict__)
    views = cpi.resample_views(to_dev(gam32), geo, ls)
    torch.cuda.synchronize()
    v = views.cpu().numpy().reshape(s.ny * s.nx, g.ha, g.wa).astype(np.float64)
    ref = oracle.refocus_resampled(gam32.astype(np.float64), g, s, [1.0])[0]
    assert np.allclose(v.sum(axis=0), ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
    gs = cpi.lens_sampling_geometry(geo, ls)
    assert (gs.wb, gs.hb) == (5, 3)
    assert np.isclose(gs.mag_x, g.mag_x * 0.7) and np.isclose(gs.cb_y, (g.cb_y + 0.5) / 1.5)


def test_paper_like_sampled_pixels(cpi):
    """Da 128 x 128, Db 64 x 64 (Gamma 16384 x 4096), lens plane oversampled 2x
    (127 x 127 samples), 32 planes; 48 output pixels of 4 planes checked
    against the oracle evaluated pixel by pixel."""
    import torch
    g = oracle.default_geometry(128, 128, 64, 64)
    rng = np.random.default_rng(7)
    gam32 = (rng.standard_normal(g.wa * g.ha * g.wb * g.hb) * 1e-3).astype(np.float32)
    s = oracle.LensSampling(127, 127, 0.0, 0.0, 0.5, 0.5)
    alphas = np.linspace(0.5, 1.5, 32)
    log("paper-like resampled refocus")
    got = _run(cpi, gam32, g, s, alphas)
    assert np.isfinite(got).all()
    ys = rng.integers(0, g.out_h, 48)
    xs = rng.integers(0, g.out_w, 48)
    planes = [0, 9, 22, 31]
    ref = oracle.refocus_resampled_pixels(gam32.astype(np.float64), g, s, alphas[planes], ys, xs)
    for k, p in enumerate(planes):
        gp = got[p, ys, xs]
        scale = max(np.abs(got[p]).max(), np.abs(ref[k]).max())
        err = np.abs(gp - ref[k]).max() / scale
        log(f"  plane {p}: sampled rel err {err:.2e}")
        assert err <= TOL
