"""GPU parity of refocusing (batched, plain and autotuned) against the FP64
oracle.  Tolerance: per plane, max |I_gpu - I_oracle| / max |I_oracle|
<= 1e-5, with I_oracle computed from the oracle's FP64 Gamma."""
import json
import os

import numpy as np
import pytest

import oracle
from synth import WORKLOADS, alphas_for, generate_frames
from tests.gpu_util import dev, log, plane_rel_err, to_dev
from tests.phantoms import point_gamma

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-5


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def assert_r12(got, want, what):
    """Per plane max |I_gpu - I_oracle| / max |I_oracle| <= 1e-5; a plane the
    oracle finds exactly zero (every sample outside the views) must be zero."""
    err = np.abs(got - want).max(axis=(1, 2))
    scale = np.abs(want).max(axis=(1, 2))
    zero = scale == 0
    assert (err[zero] == 0).all(), (what, "nonzero plane where the oracle is zero")
    rel = err[~zero] / scale[~zero]
    log(f"{what}: worst plane relative error {rel.max() if rel.size else 0.0:.3g}")
    assert (rel <= TOL).all(), (what, rel)


def _geom(cpi, g: oracle.Geometry):
    return cpi.make_geometry(**g.__dict__)


def _run(cpi, fn, gamma_vm_f32, g: oracle.Geometry, alphas):
    import torch

    out = torch.full((len(alphas) * g.out_h * g.out_w,), np.nan, dtype=torch.float32,
                     device=dev())
    fn(to_dev(np.asarray(gamma_vm_f32, dtype=np.float32)), _geom(cpi, g), alphas, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(alphas), g.out_h, g.out_w)


@pytest.mark.parametrize("path", ["batched", "plain"])
def test_hand_worked_1d(cpi, path):
    with open(os.path.join(GOLDEN, "refocus_hand_1d.json")) as f:
        fx = json.load(f)
    g = oracle.Geometry(**fx["geometry"])
    fn = cpi.refocus if path == "batched" else cpi.refocus_plain
    log(f"case hand-worked 1d {path}")
    got = _run(cpi, fn, np.array(fx["gamma_view_major"]), g, fx["alphas"])
    assert np.array_equal(got, np.array(fx["expected"], dtype=np.float32))


@pytest.fixture(scope="module")
def tiny(cpi):
    w = WORKLOADS["da32_db16_n1000_u8counts"]
    a, b = generate_frames(w, workers=1)
    ref = oracle.correlation(a, b, w.n_frames, w.pa, w.pb, oracle.FRAMES_U8)
    gvm64 = oracle.to_layout(ref["gamma"], oracle.GAMMA_VIEW_MAJOR)
    gvm32 = oracle.to_layout(ref["gamma_f32"], oracle.GAMMA_VIEW_MAJOR)
    return w, gvm64, gvm32


@pytest.mark.parametrize("path", ["batched", "plain"])
def test_tiny_workload(cpi, tiny, path):
    w, g64, g32 = tiny
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = alphas_for(w)
    fn = cpi.refocus if path == "batched" else cpi.refocus_plain
    log(f"case {w.name} refocus {path}")
    got = _run(cpi, fn, g32, g, al)
    want = oracle.refocus(g64, g, al)
    assert plane_rel_err(got, want).max() <= TOL
    again = _run(cpi, fn, g32, g, al)
    assert np.array_equal(got, again)


GEOMS = [
    # non-default centres and magnification, output grid larger than Da
    oracle.Geometry(24, 20, 6, 5, 1.7, 2.3, 10.2, 9.9, 2.4, 1.6, 70, 33),
    # output smaller than Da, tiny lens grid
    oracle.Geometry(40, 36, 3, 2, 3.0, 4.0, 19.5, 17.5, 1.0, 0.5, 17, 9),
    # minimal views
    oracle.Geometry(65, 2, 1, 1, 1.0, 1.0, 32.0, 0.5, 0.0, 0.0, 65, 2),
]
ALPHAS = [[1.0], [0.5, 0.75, 1.0, 1.25, 1.5], [-1.3, 0.0, 0.37, 2.9, 4.0, 1.0, 1.0 + 1e-9],
          list(np.linspace(0.3, 1.7, 19))]


@pytest.mark.parametrize("gi", range(len(GEOMS)))
@pytest.mark.parametrize("ai", range(len(ALPHAS)))
def test_geometries_and_alphas(cpi, gi, ai):
    g = GEOMS[gi]
    al = ALPHAS[ai]
    rng = np.random.default_rng(gi * 10 + ai)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    gam32 = gam.astype(np.float32)
    want = oracle.refocus(gam32.astype(np.float64), g, al)
    for path, fn in [("batched", cpi.refocus), ("plain", cpi.refocus_plain)]:
        log(f"case geometry {gi} alphas {ai} {path}")
        got = _run(cpi, fn, gam32, g, al)
        assert_r12(got, want, (path, gi, ai))


def test_alpha_one_row_sums(cpi, tiny):
    w, g64, g32 = tiny
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    log("case alpha=1 row sums")
    got = _run(cpi, cpi.refocus, g32, g, [1.0])[0]
    want = g64.sum(axis=0).reshape(w.ha, w.wa)
    assert plane_rel_err(got[None], want[None]).max() <= TOL


@pytest.mark.parametrize("alpha_star", [0.6, 0.75, 1.25])
def test_point_phantom(cpi, alpha_star):
    g = oracle.default_geometry(32, 32, 16, 16)
    gam, peak = point_gamma(g, alpha_star, 14, 17)
    log(f"case point phantom {alpha_star}")
    got = _run(cpi, cpi.refocus, gam, g, [alpha_star])[0]
    assert abs(got[17, 14] - peak) <= 1e-5 * peak
    assert np.unravel_index(np.argmax(got), got.shape) == (17, 14)


def test_autotune_configs_deterministic_and_accurate(cpi, tiny):
    """Every configuration the autotuner may pick meets the tolerance and is
    bitwise reproducible; the tuned call leaves a valid stack in out."""
    import torch

    w, g64, g32 = tiny
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = np.linspace(0.5, 1.5, 13)
    want = oracle.refocus(g64, g, al)
    log("case autotune")
    got = _run(cpi, cpi.autotune_refocus, g32, g, al)
    assert plane_rel_err(got, want).max() <= TOL
    after = _run(cpi, cpi.refocus, g32, g, al)   # uses the cached configuration
    assert plane_rel_err(after, want).max() <= TOL
    assert np.array_equal(after, _run(cpi, cpi.refocus, g32, g, al))
    del torch


TILE_SHAPES = [(4, 8), (4, 16), (8, 8), (8, 16), (8, 32), (16, 8), (16, 16)]
SEP_ONLY_SHAPES = [(1, 16), (2, 16), (2, 32), (4, 32)]   # column-sum kernel only


KERNELS = [(0, 0), (1, 2), (1, 3), (1, 4)]   # (kernel, copy stages)
# (8 planes x 32 rows with 4 staged windows would need more LDS than a CU has)
CONFIGS = [(shape, k) for shape in TILE_SHAPES for k in KERNELS
           if (shape, k) != ((8, 32), (1, 4))] + \
    [(shape, k) for shape in SEP_ONLY_SHAPES for k in KERNELS[1:]]


@pytest.mark.parametrize("shape,kernel", CONFIGS)
def test_every_tile_config(cpi, tiny, shape, kernel):
    """Both batched kernels (per-row interpolation; column sums over x_b
    first, with 2, 3 and 4 staged view windows) in every built tile shape and
    with 1, 2 and 5 view-row splits: within the tolerance of the oracle and
    bitwise reproducible."""
    w, g64, g32 = tiny
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = np.linspace(0.5, 1.5, 13)
    want = oracle.refocus(g64, g, al)
    kp, rw = shape
    for splits in (1, 2, 5):
        tiles = (kp, rw, splits) + kernel
        log(f"case tiles {tiles}")
        fn = lambda gam, geo, a, out: cpi.refocus_tiled(gam, geo, a, out, tiles)  # noqa: E731
        got = _run(cpi, fn, g32, g, al)
        assert plane_rel_err(got, want).max() <= TOL, tiles
        assert np.array_equal(got, _run(cpi, fn, g32, g, al)), tiles


WINDOW_GEOMS = [
    # views wider than the 128-float LDS rows: at |alpha| >= 2 the column
    # windows do not fit and the kernels gather directly from Gamma
    oracle.Geometry(136, 40, 4, 3, 2.0, 2.0, 67.5, 19.5, 1.5, 1.0, 136, 40),
    # view rows not a multiple of 4 floats (4-byte window copies); tall
    # row windows at large alpha
    oracle.Geometry(30, 53, 5, 3, 1.7, 2.3, 14.5, 26.0, 2.0, 1.0, 30, 53),
]
WINDOW_ALPHAS = [2.6, -0.8, 1.0, 0.5, 1.5, 0.0, 1.9]


@pytest.fixture(scope="module")
def window_cases():
    cases = []
    for gi, g in enumerate(WINDOW_GEOMS):
        rng = np.random.default_rng(100 + gi)
        gam32 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa)).astype(np.float32)
        want = oracle.refocus(gam32.astype(np.float64), g, WINDOW_ALPHAS)
        cases.append((g, gam32, want))
    return cases


@pytest.mark.parametrize("shape,kernel", CONFIGS)
def test_tile_configs_window_paths(cpi, window_cases, shape, kernel):
    """Every tile shape of both kernels where some windows do not fit in LDS
    (wide views, large |alpha|) and where view rows are not a multiple of 4
    floats; one and three view-row splits."""
    kp, rw = shape
    for gi, (g, gam32, want) in enumerate(window_cases):
        for splits in (1, 3):
            tiles = (kp, rw, splits) + kernel
            log(f"case window geometry {gi} tiles {tiles}")
            fn = lambda gam, geo, a, out: cpi.refocus_tiled(gam, geo, a, out, tiles)  # noqa: E731
            got = _run(cpi, fn, gam32, g, WINDOW_ALPHAS)
            assert_r12(got, want, (gi, tiles))


def test_tiles_query_and_unsupported(cpi, tiny):
    """refocus_tiles reports a built configuration; an unbuilt one is
    rejected before any launch."""
    w, _, g32 = tiny
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    kp, rw, sp, kernel, stages = cpi.refocus_tiles(_geom(cpi, g), 5)
    assert ((kp, rw), (kernel, stages)) in CONFIGS and 1 <= sp <= 16
    for bad in [(16, 32, 1, 0, 0), (8, 16, 0, 1, 3), (8, 16, 1, 3, 3), (2, 8, 1, 0, 0),
                (2, 8, 1, 2, 0), (16, 32, 1, 2, 0),
                (8, 16, 1, 1, 1), (8, 16, 1, 1, 5), (2, 16, 1, 0, 0), (1, 32, 1, 1, 2),
                (8, 32, 1, 1, 4)]:
        fn = lambda gam, geo, a, out: cpi.refocus_tiled(gam, geo, a, out, bad)  # noqa: E731
        with pytest.raises(cpi.CpiError):
            _run(cpi, fn, g32, g, [1.0])


@pytest.fixture(scope="module")
def paper_gamma():
    """Gamma of the 20000-frame paper-like workload from the oracle's exact
    correlation, view-major, FP64 and its FP32 rounding."""
    w = WORKLOADS["da128_db64_n20000_u8bin"]
    a, b = generate_frames(w)
    log(f"case {w.name} oracle Gamma")
    ref = oracle.correlation(a, b, w.n_frames, w.pa, w.pb, oracle.FRAMES_U8)
    g64 = oracle.to_layout(ref["gamma"], oracle.GAMMA_VIEW_MAJOR)
    g32 = oracle.to_layout(ref["gamma_f32"], oracle.GAMMA_VIEW_MAJOR)
    return w, g64, g32


def test_paper_like_full_size(cpi, paper_gamma):
    """Da 128x128, Db 64x64, 32 planes, Gamma from the oracle's exact
    correlation of the 20000-frame workload; checked at 96 sampled pixels of
    every plane (including each plane's largest-magnitude pixel)."""
    w, g64, g32 = paper_gamma
    log(f"case {w.name} refocus, 32 planes")
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = alphas_for(w)
    got = _run(cpi, cpi.refocus, g32, g, al)
    rng = np.random.default_rng(3)
    ys = list(rng.integers(0, w.ha, 64)) + [0, w.ha - 1, 0, w.ha - 1]
    xs = list(rng.integers(0, w.wa, 64)) + [0, 0, w.wa - 1, w.wa - 1]
    flat = np.abs(got.reshape(len(al), -1))
    for k in range(len(al)):
        yy, xx = np.unravel_index(np.argmax(flat[k]), (w.ha, w.wa))
        ys.append(yy)
        xs.append(xx)
    ys, xs = np.array(ys), np.array(xs)
    want = oracle.refocus_pixels(g64, g, al, ys, xs)
    err = plane_rel_err(got[:, ys, xs], want)
    log(f"per-plane relative error max {err.max():.3g}")
    assert err.max() <= TOL
    plain = _run(cpi, cpi.refocus_plain, g32, g, al)
    assert plane_rel_err(plain[:, ys, xs], want).max() <= TOL
    for tiles in [(8, 16, 4, 1, 3), (16, 16, 2, 1, 4), (8, 32, 2, 1, 2), (4, 8, 8, 1, 3),
                  (4, 16, 16, 1, 2), (2, 32, 16, 1, 3), (1, 16, 8, 1, 4), (8, 16, 4, 0, 0)]:
        log(f"case {w.name} refocus, 32 planes, tiles {tiles}")
        fn = lambda gam, geo, a, out: cpi.refocus_tiled(gam, geo, a, out, tiles)  # noqa: E731
        got_t = _run(cpi, fn, g32, g, al)
        err = plane_rel_err(got_t[:, ys, xs], want)
        log(f"tiles {tiles}: per-plane relative error max {err.max():.3g}")
        assert err.max() <= TOL, tiles


@pytest.mark.parametrize("n_alpha", [100, 261, 1000])
def test_paper_plane_counts(cpi, paper_gamma, n_alpha):
    """The paper's stack sizes (100, 261 and 1000 planes, alpha in [0.5, 1.5])
    in one call each at the paper-like geometry: 24 evenly spaced planes
    (first and last included) checked at 64 sampled pixels plus each checked
    plane's largest-magnitude pixel."""
    w, g64, g32 = paper_gamma
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = np.linspace(0.5, 1.5, n_alpha)
    log(f"case {w.name} refocus, {n_alpha} planes")
    got = _run(cpi, cpi.refocus, g32, g, al)
    assert np.isfinite(got).all()
    planes = np.unique(np.linspace(0, n_alpha - 1, 24).round().astype(int))
    rng = np.random.default_rng(n_alpha)
    ys = list(rng.integers(0, w.ha, 64))
    xs = list(rng.integers(0, w.wa, 64))
    flat = np.abs(got[planes].reshape(planes.size, -1))
    for k in range(planes.size):
        yy, xx = np.unravel_index(np.argmax(flat[k]), (w.ha, w.wa))
        ys.append(yy)
        xs.append(xx)
    ys, xs = np.array(ys), np.array(xs)
    want = oracle.refocus_pixels(g64, g, al[planes], ys, xs)
    err = plane_rel_err(got[planes][:, ys, xs], want)
    log(f"{n_alpha} planes: per-plane relative error max {err.max():.3g}")
    assert err.max() <= TOL
