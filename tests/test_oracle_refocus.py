"""Pins of the refocusing oracle (CPU only).

The oracle is tied to: a hand-worked example; the general 4-D multilinear
interpolation of Gamma evaluated in exact rational arithmetic; the alpha = 1
and alpha = 0 closed forms; an integer-geometry shear-and-sum; exact
reproduction of affine data; linearity; and point phantoms whose focal plane
and position are known (closed-form Gamma and simulated frames).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import Geometry, default_geometry
from tests.phantoms import point_frames, point_gamma

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_1d():
    with open(os.path.join(GOLDEN, "refocus_hand_1d.json")) as f:
        fx = json.load(f)
    g = Geometry(**fx["geometry"])
    got = oracle.refocus(np.array(fx["gamma_view_major"], dtype=np.float64), g, fx["alphas"])
    assert np.array_equal(got, np.array(fx["expected"], dtype=np.float64))


def _multilinear_4d_fraction(gam_vm, g, alpha, xr, yr):
    """Exact 4-D multilinear interpolation of Gamma(x, y, x_b, y_b), summed over
    the integer lens-plane grid.  The (x_b, y_b) coordinates of the sample are
    integers, so their weights are 1 on the grid point and 0 on its neighbour;
    the loop still visits all 16 corners to check that reduction."""
    a = Fraction(alpha)
    total = Fraction(0)
    gv = gam_vm.reshape(g.hb, g.wb, g.ha, g.wa)

    def val(x, y, xb, yb):
        if 0 <= x < g.wa and 0 <= y < g.ha and 0 <= xb < g.wb and 0 <= yb < g.hb:
            return Fraction(gv[yb, xb, y, x])
        return Fraction(0)

    for yb in range(g.hb):
        for xb in range(g.wb):
            ux = a * (xr - Fraction(g.ca_x)) + Fraction(g.ca_x) + (1 - a) * Fraction(g.mag_x) * (xb - Fraction(g.cb_x))
            uy = a * (yr - Fraction(g.ca_y)) + Fraction(g.ca_y) + (1 - a) * Fraction(g.mag_y) * (yb - Fraction(g.cb_y))
            pts = [ux, uy, Fraction(xb), Fraction(yb)]
            lo = [math.floor(p) for p in pts]
            fr = [p - l for p, l in zip(pts, lo)]
            for corner in range(16):
                w = Fraction(1)
                idx = []
                for d in range(4):
                    bit = (corner >> d) & 1
                    w *= fr[d] if bit else 1 - fr[d]
                    idx.append(lo[d] + bit)
                if w:
                    total += w * val(*idx)
    return total


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.77, 1.0, 1.25, 1.5, -0.4, 2.6])
def test_bruteforce_multilinear_fraction(alpha):
    g = Geometry(5, 4, 3, 2, 1.7, 2.0, 2.1, 1.5, 1.0, 0.25, 6, 5)
    rng = np.random.default_rng(int(abs(alpha) * 100) + 7)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    got = oracle.refocus(gam, g, [alpha])[0]
    scale = np.abs(gam).sum()
    for yr in range(g.out_h):
        for xr in range(g.out_w):
            want = float(_multilinear_4d_fraction(gam, g, alpha, xr, yr))
            assert abs(got[yr, xr] - want) <= 1e-13 * scale


def test_alpha_one_is_row_sum_of_numerator():
    """alpha = 1: each output pixel is the row sum of Gamma over rho_b, which
    equals (N sum_i A_i[p] |B_i| - S_a[p] sum S_b) / N^2 from the frames."""
    rng = np.random.default_rng(12)
    wa, ha, wb, hb, n = 12, 10, 6, 5, 400
    a = rng.integers(0, 5, size=(n, wa * ha)).astype(np.uint8)
    b = rng.integers(0, 5, size=(n, wb * hb)).astype(np.uint8)
    r = oracle.correlation(a, b, n, wa * ha, wb * hb, oracle.FRAMES_U8)
    g = default_geometry(wa, ha, wb, hb)
    out = oracle.refocus(oracle.to_layout(r["gamma"], oracle.GAMMA_VIEW_MAJOR), g, [1.0])[0]
    a64, b64 = a.astype(np.int64), b.astype(np.int64)
    rows = n * (a64 * b64.sum(axis=1)[:, None]).sum(axis=0) - a64.sum(axis=0) * b64.sum()
    want = (rows / float(n * n)).reshape(ha, wa)
    assert np.allclose(out, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_alpha_zero_is_constant():
    g = default_geometry(16, 12, 8, 6)
    rng = np.random.default_rng(13)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    out = oracle.refocus(gam, g, [0.0])[0]
    assert np.ptp(out) <= 1e-12 * np.abs(out).max()


@pytest.mark.parametrize("alpha", [-1, 0, 1, 2, 3])
def test_integer_geometry_shear_and_sum(alpha):
    """c = 0, M = 1, integer alpha: every sample point is a grid point, so the
    refocus is a pure gather ("shift and sum") with zeros outside the view."""
    wa, ha, wb, hb = 9, 7, 4, 3
    g = Geometry(wa, ha, wb, hb, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0, wa, ha)
    rng = np.random.default_rng(14 + alpha + 1)
    gam = rng.integers(-50, 50, size=(hb * wb, ha * wa)).astype(np.float64)
    got = oracle.refocus(gam, g, [float(alpha)])[0]
    want = np.zeros((ha, wa))
    for yr in range(ha):
        for xr in range(wa):
            for yb in range(hb):
                for xb in range(wb):
                    x = alpha * xr + (1 - alpha) * xb
                    y = alpha * yr + (1 - alpha) * yb
                    if 0 <= x < wa and 0 <= y < ha:
                        want[yr, xr] += gam[yb * wb + xb, y * wa + x]
    assert np.array_equal(got, want)


def test_affine_data_reproduced_exactly():
    """Bilinear interpolation reproduces affine views: with
    Gamma(x, y; rho_b) = s*x + t*y + c(rho_b), interior samples give
    I = sum_b (s*u_x + t*u_y + c(rho_b)), summed here in closed form."""
    g = Geometry(40, 36, 6, 5, 1.5, 1.25, 20.3, 17.1, 2.2, 1.9, 40, 36)
    s, t = 0.37, -1.21
    rng = np.random.default_rng(15)
    c = rng.standard_normal(g.hb * g.wb)
    xs = np.arange(g.wa, dtype=np.float64)
    ys = np.arange(g.ha, dtype=np.float64)
    view = s * xs[None, :] + t * ys[:, None]
    gam = np.stack([(view + c[k]).reshape(-1) for k in range(g.hb * g.wb)])
    for alpha in [0.8, 0.93, 1.0, 1.1]:
        out = oracle.refocus(gam, g, [alpha])[0]
        pb = g.hb * g.wb
        sum_bx = (1 - alpha) * g.mag_x * g.hb * (g.wb * (g.wb - 1) / 2.0 - g.wb * g.cb_x)
        sum_by = (1 - alpha) * g.mag_y * g.wb * (g.hb * (g.hb - 1) / 2.0 - g.hb * g.cb_y)
        for yr in range(12, 24):
            for xr in range(12, 28):
                ax = alpha * (xr - g.ca_x) + g.ca_x
                ay = alpha * (yr - g.ca_y) + g.ca_y
                want = s * (pb * ax + sum_bx) + t * (pb * ay + sum_by) + c.sum()
                assert abs(out[yr, xr] - want) < 1e-11 * (1 + abs(want))


def test_linearity():
    g = default_geometry(14, 10, 7, 5)
    rng = np.random.default_rng(16)
    g1 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    g2 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    al = [0.6, 1.0, 1.3]
    lhs = oracle.refocus(2.5 * g1 - 0.75 * g2, g, al)
    rhs = 2.5 * oracle.refocus(g1, g, al) - 0.75 * oracle.refocus(g2, g, al)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)


def test_pixel_list_matches_grid():
    g = default_geometry(16, 16, 8, 8)
    rng = np.random.default_rng(17)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    al = [0.55, 1.45]
    full = oracle.refocus(gam, g, al)
    ys = np.array([0, 3, 15, 8])
    xs = np.array([0, 15, 7, 8])
    part = oracle.refocus_pixels(gam, g, al, ys, xs)
    assert np.array_equal(part, full[:, ys, xs])


@pytest.mark.parametrize("alpha_star", [0.6, 0.75, 0.9, 1.25])
def test_point_phantom_closed_form(alpha_star):
    g = default_geometry(32, 32, 16, 16)
    xo, yo = 14, 17
    gam, peak = point_gamma(g, alpha_star, xo, yo)
    out = oracle.refocus(gam, g, [alpha_star])[0]
    assert abs(out[yo, xo] - peak) < 1e-12 * peak
    assert np.unravel_index(np.argmax(out), out.shape) == (yo, xo)
    # focal-plane search on a 0.01 grid: bilinear blur biases it by <= one step
    grid = np.round(np.arange(alpha_star - 0.1, alpha_star + 0.1001, 0.01), 10)
    stack = oracle.refocus(gam, g, grid)
    best = grid[np.argmax(stack.reshape(grid.size, -1).max(axis=1))]
    assert abs(best - alpha_star) <= 0.0100001


def test_point_phantom_integer_geometry_reaches_pb():
    g = Geometry(16, 16, 4, 4, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 16, 16)
    gam, peak = point_gamma(g, 2.0, 6, 7)
    assert peak == g.wb * g.hb
    out = oracle.refocus(gam, g, [2.0])[0]
    assert out[7, 6] == g.wb * g.hb
    assert out.sum() == g.wb * g.hb


def test_point_object_frames_end_to_end():
    """Frames of a point object at alpha* = 0.75: Gamma estimated from 2e4
    frames, refocused, peaks at the object pixel and the best plane."""
    g = default_geometry(32, 32, 16, 16)
    alpha_star, xo, yo = 0.75, 13, 18
    a, b = point_frames(g, alpha_star, xo, yo, 20000, 1.0, seed=18)
    r = oracle.correlation(a, b, a.shape[0], g.wa * g.ha, g.wb * g.hb, oracle.FRAMES_U8)
    gam = oracle.to_layout(r["gamma"], oracle.GAMMA_VIEW_MAJOR)
    out = oracle.refocus(gam, g, [alpha_star])[0]
    assert np.unravel_index(np.argmax(out), out.shape) == (yo, xo)
    grid = np.round(np.arange(0.6, 0.9001, 0.01), 10)
    stack = oracle.refocus(gam, g, grid)
    best = grid[np.argmax(stack.reshape(grid.size, -1).max(axis=1))]
    assert abs(best - alpha_star) <= 0.02 + 1e-9


# ---- resampled lens-plane grid (general 4-D multilinear interpolation) -------------
def _multilinear_4d_fraction_sampled(gam_vm, g, s, alpha, xr, yr):
    """Exact 4-D multilinear interpolation of Gamma at every lens-plane sample
    point (fractional x_b, y_b), summed over the samples."""
    a = Fraction(alpha)
    gv = gam_vm.reshape(g.hb, g.wb, g.ha, g.wa)

    def val(x, y, xb, yb):
        if 0 <= x < g.wa and 0 <= y < g.ha and 0 <= xb < g.wb and 0 <= yb < g.hb:
            return Fraction(gv[yb, xb, y, x])
        return Fraction(0)

    total = Fraction(0)
    for j in range(s.ny):
        for i in range(s.nx):
            xb = Fraction(s.ox) + i * Fraction(s.sx)
            yb = Fraction(s.oy) + j * Fraction(s.sy)
            ux = a * (xr - Fraction(g.ca_x)) + Fraction(g.ca_x) + (1 - a) * Fraction(g.mag_x) * (xb - Fraction(g.cb_x))
            uy = a * (yr - Fraction(g.ca_y)) + Fraction(g.ca_y) + (1 - a) * Fraction(g.mag_y) * (yb - Fraction(g.cb_y))
            pts = [ux, uy, xb, yb]
            lo = [math.floor(p) for p in pts]
            fr = [p - l for p, l in zip(pts, lo)]
            for corner in range(16):
                w = Fraction(1)
                idx = []
                for d in range(4):
                    bit = (corner >> d) & 1
                    w *= fr[d] if bit else 1 - fr[d]
                    idx.append(lo[d] + bit)
                if w:
                    total += w * val(*idx)
    return total


@pytest.mark.parametrize("alpha", [0.4, 0.77, 1.0, 1.3, 2.2])
def test_resampled_bruteforce_fraction(alpha):
    g = Geometry(5, 4, 3, 3, 1.7, 1.3, 2.1, 1.5, 1.0, 1.25, 5, 4)
    s = oracle.LensSampling(4, 3, -0.25, 0.5, 0.75, 0.625)
    rng = np.random.default_rng(int(abs(alpha) * 100) + 11)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    got = oracle.refocus_resampled(gam, g, s, [alpha])[0]
    scale = np.abs(gam).sum()
    for yr in range(g.out_h):
        for xr in range(g.out_w):
            want = float(_multilinear_4d_fraction_sampled(gam, g, s, alpha, xr, yr))
            assert abs(got[yr, xr] - want) <= 1e-13 * scale
    pix = oracle.refocus_resampled_pixels(gam, g, s, [alpha], [0, 3, 2], [4, 1, 2])[0]
    assert np.allclose(pix, [got[0, 4], got[3, 1], got[2, 2]], rtol=0, atol=1e-14 * scale)


def test_resampled_integer_grid_is_refocus():
    g = default_geometry(12, 10, 6, 5)
    rng = np.random.default_rng(12)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    s = oracle.LensSampling(g.wb, g.hb, 0.0, 0.0, 1.0, 1.0)
    al = [0.5, 0.9, 1.0, 1.45]
    assert np.allclose(oracle.refocus_resampled(gam, g, s, al), oracle.refocus(gam, g, al),
                       rtol=1e-13, atol=1e-13)


def test_resampled_half_step_alpha_one_closed_form():
    """alpha = 1 puts every sample at u = output pixel, so each view enters with
    the total weight of the samples around it: on the grid 0, 0.5, ..., W_b - 1
    that is 2 for inner views and 1.5 for the two end views, per axis."""
    g = default_geometry(8, 6, 4, 3)
    rng = np.random.default_rng(13)
    gam = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    s = oracle.LensSampling(2 * g.wb - 1, 2 * g.hb - 1, 0.0, 0.0, 0.5, 0.5)
    wx = np.full(g.wb, 2.0)
    wx[[0, -1]] = 1.5
    wy = np.full(g.hb, 2.0)
    wy[[0, -1]] = 1.5
    views = gam.reshape(g.hb, g.wb, g.ha, g.wa)
    want = np.einsum("j,i,jiyx->yx", wy, wx, views)
    got = oracle.refocus_resampled(gam, g, s, [1.0])[0]
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_resampled_reproduces_multilinear_data():
    """Gamma sampled from a function affine in each of its four coordinates is
    reproduced exactly by the interpolation wherever all 16 corners lie inside
    both detectors, so the stack is the sum of that function over the samples."""
    g = Geometry(20, 18, 6, 5, 2.0, 2.0, 9.5, 8.5, 2.5, 2.0, 20, 18)
    c = np.array([0.3, -0.2, 0.5, 1.1, 0.7])

    def f(x, y, xb, yb):
        return (c[0] + c[1] * x) * (1.0 + 0.05 * y) * (c[2] + c[3] * xb) * (c[4] + 0.1 * yb)

    yy, xx = np.mgrid[0:g.ha, 0:g.wa]
    gam = np.stack([f(xx, yy, xb, yb) for yb in range(g.hb) for xb in range(g.wb)])
    s = oracle.LensSampling(5, 4, 0.5, 0.25, 0.875, 0.9)   # inside [0, 4] x [0, 3.7]
    alpha = 0.9
    got = oracle.refocus_resampled(gam.reshape(g.hb * g.wb, -1), g, s, [alpha])[0]
    for yr in range(6, 12):
        for xr in range(6, 14):
            want = 0.0
            for j in range(s.ny):
                for i in range(s.nx):
                    xb, yb = s.ox + i * s.sx, s.oy + j * s.sy
                    ux = alpha * (xr - g.ca_x) + g.ca_x + (1 - alpha) * g.mag_x * (xb - g.cb_x)
                    uy = alpha * (yr - g.ca_y) + g.ca_y + (1 - alpha) * g.mag_y * (yb - g.cb_y)
                    want += f(ux, uy, xb, yb)
            assert abs(got[yr, xr] - want) <= 1e-12 * abs(want) + 1e-12


def test_resampled_linearity():
    g = default_geometry(8, 8, 4, 4)
    rng = np.random.default_rng(14)
    g1 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    g2 = rng.standard_normal((g.hb * g.wb, g.ha * g.wa))
    s = oracle.LensSampling(5, 6, -0.3, 0.2, 0.8, 0.6)
    al = [0.6, 1.2]
    lhs = oracle.refocus_resampled(2.0 * g1 - 3.0 * g2, g, s, al)
    rhs = 2.0 * oracle.refocus_resampled(g1, g, s, al) - 3.0 * oracle.refocus_resampled(g2, g, s, al)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_default_geometry_values():
    """Default geometry: magnification Wa/Wb and Ha/Hb, centres at (W - 1)/2
    on both detectors, output on detector A's grid."""
    g = default_geometry(128, 96, 64, 32)
    assert (g.wa, g.ha, g.wb, g.hb) == (128, 96, 64, 32)
    assert (g.mag_x, g.mag_y) == (2.0, 3.0)
    assert (g.ca_x, g.ca_y, g.cb_x, g.cb_y) == (63.5, 47.5, 31.5, 15.5)
    assert (g.out_w, g.out_h) == (128, 96)
    g = default_geometry(7, 5, 3, 2)
    assert (g.mag_x, g.mag_y) == (7 / 3, 2.5)
    assert (g.ca_x, g.ca_y, g.cb_x, g.cb_y) == (3.0, 2.0, 1.0, 0.5)
