"""GPU parity of the row-lane refocus kernel (lanes are view rows; column
sums over x_b written per (plane, y_b), then folded over y_b) against the
FP64 oracle, graded per plane by max |I_gpu - I_oracle| / max |I_oracle|
<= 1e-5 on a seeded random FP32 Gamma."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import log, plane_rel_err
from tests.test_gpu_refocus import TOL, _geom, _run, assert_r12

pytestmark = pytest.mark.gpu

ROWS_SHAPES = [(8, 8), (4, 16), (8, 16), (16, 16), (8, 32)]

# (geometry, alphas): one, two and four row waves, a partial last row wave,
# output grids other than the detector-A grid (ragged output columns), and
# plane counts that are not a multiple of the planes per work-group
CASES = [
    (oracle.Geometry(64, 48, 16, 12, 4.0, 4.0, 31.5, 23.5, 7.5, 5.5, 64, 48),
     np.linspace(0.5, 1.5, 13)),
    (oracle.Geometry(96, 128, 8, 8, 2.0, 2.0, 47.5, 63.5, 3.5, 3.5, 90, 120),
     np.linspace(0.7, 1.3, 21)),
    (oracle.Geometry(72, 200, 6, 10, 1.5, 2.0, 35.5, 99.5, 2.5, 4.5, 70, 203),
     np.array([1.0, 0.6, 1.2, 0.95, 1.05, 0.8, 1.4, 0.5, 1.1])),
    (oracle.Geometry(80, 256, 5, 4, 2.0, 2.0, 39.5, 127.5, 2.0, 1.5, 80, 256),
     np.linspace(0.5, 1.5, 19)),
]


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


@pytest.fixture(scope="module")
def cases():
    out = []
    for i, (g, al) in enumerate(CASES):
        rng = np.random.default_rng(500 + i)
        gam32 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa)).astype(np.float32)
        want = oracle.refocus(gam32.astype(np.float64), g, al)
        out.append((g, al, gam32, want))
    return out


def _tiled(cpi, tiles):
    return lambda gam, geo, a, out: cpi.refocus_tiled(gam, geo, a, out, tiles)  # noqa: E731


@pytest.mark.parametrize("shape", ROWS_SHAPES)
def test_rows_shapes(cpi, cases, shape):
    """Every built (planes, output columns) shape on every case where its
    staged window holds the plane groups' sample columns; bitwise
    reproducible; a case it does not take is rejected before any launch."""
    ran = 0
    for i, (g, al, gam32, want) in enumerate(cases):
        tiles = (shape[0], shape[1], 1, cpi.REFOCUS_VIEW_ROWS, 0)
        log(f"case rows {i} tiles {tiles}")
        fn = _tiled(cpi, tiles)
        try:
            got = _run(cpi, fn, gam32, g, al)
        except cpi.CpiError as e:
            assert e.status == 2, e   # CPI_ERR_UNSUPPORTED
            log(f"case rows {i} tiles {tiles}: not taken")
            continue
        ran += 1
        assert_r12(got, want, (i, tiles))
        assert np.array_equal(got, _run(cpi, fn, gam32, g, al)), (i, tiles)
    assert ran >= 2, shape


def test_rows_rejects_wide_plane_sets(cpi, cases):
    """A plane set whose sample columns are too wide for the staged windows
    (|alpha| up to 3) is rejected before any launch; cpi_refocus still
    refocuses it."""
    g, al, gam32, want = cases[0]
    wide = np.array([3.0, -2.0, 1.0, 0.5, 2.5, -1.0, 0.0, 1.7, 2.2])
    want_w = oracle.refocus(gam32.astype(np.float64), g, wide)
    log("case rows wide plane set")
    assert_r12(_run(cpi, cpi.refocus, gam32, g, wide), want_w, "default kernel")
    with pytest.raises(cpi.CpiError):
        _run(cpi, _tiled(cpi, (8, 8, 1, cpi.REFOCUS_VIEW_ROWS, 0)), gam32, g, wide)


def test_rows_plane_chunks(cpi, cases):
    """More planes than one chunk of the x pass's workspace (chunks of up to
    256 planes): 300 planes in one call, every plane against the oracle."""
    g, _, gam32, _ = cases[1]
    al = np.linspace(0.6, 1.4, 300)
    want = oracle.refocus(gam32.astype(np.float64), g, al)
    log("case rows 300 planes")
    got = _run(cpi, _tiled(cpi, (8, 16, 1, cpi.REFOCUS_VIEW_ROWS, 0)), gam32, g, al)
    err = plane_rel_err(got, want)
    log(f"rows 300 planes: worst plane relative error {err.max():.3g}")
    assert err.max() <= TOL


def test_rows_empty_planes(cpi):
    """Planes whose samples all fall outside the views (every weight zero)
    give exact zeros, beside ordinary planes in the same work-group."""
    g = oracle.Geometry(64, 64, 8, 8, 2.0, 2.0, 31.5, 31.5, 3.5, 3.5, 64, 64)
    rng = np.random.default_rng(77)
    gam32 = rng.standard_normal((64, 64 * 64)).astype(np.float32)
    # alpha = 1 + 200/31.5 maps every output column but the centre's outside
    al = np.array([1.0, 0.9, 1.1, 1.05, 0.95, 1.02, 0.98, 1.01])
    want = oracle.refocus(gam32.astype(np.float64), g, al)
    log("case rows ordinary planes")
    got = _run(cpi, _tiled(cpi, (8, 8, 1, cpi.REFOCUS_VIEW_ROWS, 0)), gam32, g, al)
    assert_r12(got, want, "ordinary")
    g2 = oracle.Geometry(64, 64, 8, 8, 2.0, 2.0, 200.0, 200.0, 3.5, 3.5, 64, 64)
    al2 = np.array([1.0, 1.01, 0.99, 1.02])
    want2 = oracle.refocus(gam32.astype(np.float64), g2, al2)
    log("case rows planes outside the views")
    got2 = _run(cpi, _tiled(cpi, (8, 8, 1, cpi.REFOCUS_VIEW_ROWS, 0)), gam32, g2, al2)
    assert_r12(got2, want2, "outside")
