"""The allocation-free refocus entry point (workspace in the library's fixed
per-device array) against cpi_refocus on the same inputs: bitwise equal for
the same configuration and within the refocus tolerance of the FP64 oracle,
on two calls in a row (the second smaller), with view-row splits reduced to
fit the array, and rejected before any launch when the tables alone do not
fit."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, log, plane_rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def _case(seed, g, n_alpha):
    rng = np.random.default_rng(seed)
    gam32 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa)).astype(np.float32)
    al = np.linspace(0.5, 1.5, n_alpha)
    return gam32, al


def _both(cpi, g, gam32, al, tiles=None):
    import torch

    gam = torch.from_numpy(gam32.reshape(-1)).to(dev())
    geo = cpi.make_geometry(**g.__dict__)
    n = len(al) * g.out_h * g.out_w
    out_na = torch.full((n,), np.nan, dtype=torch.float32, device=dev())
    out_ref = torch.full((n,), np.nan, dtype=torch.float32, device=dev())
    cpi.refocus_noalloc(gam, geo, al, out_na)
    if tiles is None:
        cpi.refocus(gam, geo, al, out_ref)
    else:
        cpi.refocus_tiled(gam, geo, al, out_ref, tiles)
    torch.cuda.synchronize()
    shape = (len(al), g.out_h, g.out_w)
    return out_na.cpu().numpy().reshape(shape), out_ref.cpu().numpy().reshape(shape)


def test_two_calls_second_smaller(cpi):
    """Two calls in a row on one device, the second with a smaller geometry
    and fewer planes: each meets the refocus tolerance against cpi_refocus
    (which may take the row-lane kernel, summing in another order) and
    against the oracle; where cpi_refocus takes the column-sum kernel, the
    two are equal bit for bit."""
    for seed, g, n_alpha in [
            (11, oracle.Geometry(64, 64, 16, 16, 4.0, 4.0, 31.5, 31.5, 7.5, 7.5, 64, 64), 13),
            (12, oracle.Geometry(32, 24, 8, 6, 4.0, 4.0, 15.5, 11.5, 3.5, 2.5, 30, 20), 5)]:
        log(f"case noalloc seed {seed} {g.wa}x{g.ha} views {g.wb}x{g.hb} planes {n_alpha}")
        gam32, al = _case(seed, g, n_alpha)
        got, ref = _both(cpi, g, gam32, al)
        assert plane_rel_err(got, ref).max() <= TOL
        if cpi.refocus_tiles(cpi.make_geometry(**g.__dict__), n_alpha)[3] != 2:
            assert np.array_equal(got, ref)
        want = oracle.refocus(gam32.astype(np.float64), g, al)
        err = plane_rel_err(got, want)
        log(f"noalloc seed {seed}: worst plane relative error {err.max():.3g}")
        assert err.max() <= TOL


def test_splits_reduced_to_fit(cpi):
    """200 planes at Da 128x128, Db 64x64: cpi_refocus's default is the
    row-lane kernel, which the allocation-free call replaces by the
    column-sum default (4 planes x 16 rows, 16 view-row splits, 2 staged
    windows); its partial sums need more than the 128 MiB array, so it takes
    8 splits: equal to cpi_refocus_tiled with that configuration, sampled
    pixels within the tolerance of the oracle."""
    g = oracle.default_geometry(128, 128, 64, 64)
    gam32, al = _case(13, g, 200)
    tiles = cpi.refocus_tiles(cpi.make_geometry(**g.__dict__), 200)
    if tiles[3] != 2:
        pytest.skip(f"cpi_refocus takes {tiles} here (tuned cache)")
    log("case noalloc 200 planes, splits reduced")
    got, ref = _both(cpi, g, gam32, al, tiles=(4, 16, 8, 1, 2))
    assert np.array_equal(got, ref)
    rng = np.random.default_rng(14)
    ys, xs = rng.integers(0, g.out_h, 48), rng.integers(0, g.out_w, 48)
    planes = np.array([0, 57, 99, 150, 199])
    want = oracle.refocus_pixels(gam32.astype(np.float64), g, al[planes], ys, xs)
    err = plane_rel_err(got[planes][:, ys, xs], want)
    log(f"noalloc 200 planes: worst sampled-plane relative error {err.max():.3g}")
    assert err.max() <= TOL


def test_rejects_tables_beyond_array(cpi):
    """Row tables alone above 128 MiB (4096 planes x 64 lens-plane rows x 128
    output rows x 16 bytes = 512 MiB): CPI_ERR_WORKSPACE before any launch."""
    import torch

    g = oracle.default_geometry(128, 128, 64, 64)
    geo = cpi.make_geometry(**g.__dict__)
    gam = torch.zeros(g.wa * g.ha * g.wb * g.hb, dtype=torch.float32, device=dev())
    al = np.linspace(0.5, 1.5, 4096)
    out = torch.zeros(len(al) * g.out_h * g.out_w, dtype=torch.float32, device=dev())
    with pytest.raises(cpi.CpiError) as e:
        cpi.refocus_noalloc(gam, geo, al, out)
    assert e.value.status == 4   # CPI_ERR_WORKSPACE
