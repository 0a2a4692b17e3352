"""Oracle for shift-and-sum refocusing (test infrastructure only).

The paper extracts the 3-D stack of axial sections from Gamma by a
Radon-transform based refocusing (Section "CPI algorithm", item 2) whose
prototype is a multilinear interpolation of Gamma at points that depend on the
refocusing plane (Section 4.1, refocusing optimisation).  The paper defers the
formula to its references, so this oracle takes the standard CPI reading:
every detector-B pixel rho_b selects a perspective view Gamma(., rho_b) of size
Ha x Wa; the view is resampled at a point that moves linearly with rho_b and
the samples are summed over rho_b.  For a plane parameter alpha and an output
pixel (x_r, y_r):

    u_x = alpha*(x_r - c_ax) + c_ax + (1 - alpha)*M_x*(x_b - c_bx)
    u_y = alpha*(y_r - c_ay) + c_ay + (1 - alpha)*M_y*(y_b - c_by)
    I_alpha(x_r, y_r) = sum_{y_b < Hb} sum_{x_b < Wb} bilin(Gamma(., rho_b); u_x, u_y)

where bilin takes x0 = floor(u_x), f_x = u_x - x0 (likewise in y) and sums the
four corner values weighted by (1-f_x or f_x)*(1-f_y or f_y), each corner that
falls outside [0, Wa-1] x [0, Ha-1] contributing zero.  Because rho_b runs over
its own integer grid, the multilinear interpolation in the 4-D Gamma reduces to
this bilinear one in rho_a.  alpha = 1 is the plane conjugate to detector A.

Everything is FP64; the sum over views is a plain running sum (its rounding,
at most ~Pb * 2^-53 relative, is far below any tolerance used against it).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    wa: int
    ha: int
    wb: int
    hb: int
    mag_x: float
    mag_y: float
    ca_x: float
    ca_y: float
    cb_x: float
    cb_y: float
    out_w: int
    out_h: int


def default_geometry(wa: int, ha: int, wb: int, hb: int) -> Geometry:
    """Magnification Wa/Wb and Ha/Hb, detector centres, output on the Da grid."""
    return Geometry(wa, ha, wb, hb, wa / wb, ha / hb, (wa - 1) / 2.0,
                    (ha - 1) / 2.0, (wb - 1) / 2.0, (hb - 1) / 2.0, wa, ha)


def _views(gamma_vm, g: Geometry) -> np.ndarray:
    gv = np.asarray(gamma_vm, dtype=np.float64)
    if gv.size != g.wa * g.ha * g.wb * g.hb:
        raise ValueError("gamma size does not match the geometry")
    return gv.reshape(g.hb * g.wb, g.ha, g.wa)


def _sample_sum(views, g: Geometry, alpha: float, xr: np.ndarray, yr: np.ndarray,
                grid: bool) -> np.ndarray:
    """Sum over views of the bilinear sample at the alpha-dependent points.

    ``grid``: xr, yr are the axes of a rectangular output grid (result
    len(yr) x len(xr)); otherwise they are paired pixel lists (result len(xr)).
    """
    a = float(alpha)
    ax = a * (xr - g.ca_x) + g.ca_x
    ay = a * (yr - g.ca_y) + g.ca_y
    shape = (yr.size, xr.size) if grid else (xr.size,)
    acc = np.zeros(shape, dtype=np.float64)
    for yb in range(g.hb):
        uy = ay + (1.0 - a) * g.mag_y * (yb - g.cb_y)
        y0 = np.floor(uy)
        fy = uy - y0
        y0 = y0.astype(np.int64)
        for xb in range(g.wb):
            ux = ax + (1.0 - a) * g.mag_x * (xb - g.cb_x)
            x0 = np.floor(ux)
            fx = ux - x0
            x0 = x0.astype(np.int64)
            view = views[yb * g.wb + xb]
            for dy in (0, 1):
                yy = y0 + dy
                wy = fy if dy else 1.0 - fy
                vy = (yy >= 0) & (yy < g.ha)
                yc = np.clip(yy, 0, g.ha - 1)
                for dx in (0, 1):
                    xx = x0 + dx
                    wx = fx if dx else 1.0 - fx
                    vx = (xx >= 0) & (xx < g.wa)
                    xc = np.clip(xx, 0, g.wa - 1)
                    if grid:
                        tap = view[yc[:, None], xc[None, :]]
                        tap = np.where(vy[:, None] & vx[None, :], tap, 0.0)
                        acc += (wy[:, None] * wx[None, :]) * tap
                    else:
                        tap = view[yc, xc]
                        tap = np.where(vy & vx, tap, 0.0)
                        acc += (wy * wx) * tap
    return acc


def refocus(gamma_vm, g: Geometry, alphas) -> np.ndarray:
    """Refocused stack (n_alpha, out_h, out_w) in FP64.

    ``gamma_vm`` is Gamma in view-major storage: Pb views, each Ha x Wa.
    """
    views = _views(gamma_vm, g)
    xr = np.arange(g.out_w, dtype=np.float64)
    yr = np.arange(g.out_h, dtype=np.float64)
    al = np.asarray(alphas, dtype=np.float64).reshape(-1)
    out = np.empty((al.size, g.out_h, g.out_w), dtype=np.float64)
    for k, a in enumerate(al):
        out[k] = _sample_sum(views, g, a, xr, yr, grid=True)
    return out


def refocus_pixels(gamma_vm, g: Geometry, alphas, ys, xs) -> np.ndarray:
    """The refocused values at the listed output pixels: (n_alpha, len(ys))."""
    views = _views(gamma_vm, g)
    xr = np.asarray(xs, dtype=np.float64).reshape(-1)
    yr = np.asarray(ys, dtype=np.float64).reshape(-1)
    al = np.asarray(alphas, dtype=np.float64).reshape(-1)
    out = np.empty((al.size, xr.size), dtype=np.float64)
    for k, a in enumerate(al):
        out[k] = _sample_sum(views, g, a, xr, yr, grid=False)
    return out


# ---- refocusing with a resampled lens-plane grid ------------------------------------
@dataclass(frozen=True)
class LensSampling:
    """Sample points of the detector-B (lens-plane) coordinate:
    x_b(i) = ox + i * sx (i < nx), y_b(j) = oy + j * sy (j < ny), in pixels."""
    nx: int
    ny: int
    ox: float
    oy: float
    sx: float
    sy: float


def _floor_frac(v):
    v0 = np.floor(v)
    return v0.astype(np.int64), v - v0


def _resampled_sum(views, g: Geometry, s: LensSampling, alpha: float, xr, yr, grid: bool):
    """Sum over the lens-plane sample points of the 4-D multilinear interpolant
    of Gamma at (u_x, u_y, x_b, y_b): 16 corners, each weighted by the product
    of its four linear weights, corners outside either detector contributing
    zero."""
    a = float(alpha)
    ax = a * (xr - g.ca_x) + g.ca_x
    ay = a * (yr - g.ca_y) + g.ca_y
    shape = (yr.size, xr.size) if grid else (xr.size,)
    acc = np.zeros(shape, dtype=np.float64)
    for j in range(s.ny):
        yb = s.oy + j * s.sy
        yb0, fyb = _floor_frac(np.float64(yb))
        uy = ay + (1.0 - a) * g.mag_y * (yb - g.cb_y)
        y0, fy = _floor_frac(uy)
        for i in range(s.nx):
            xb = s.ox + i * s.sx
            xb0, fxb = _floor_frac(np.float64(xb))
            ux = ax + (1.0 - a) * g.mag_x * (xb - g.cb_x)
            x0, fx = _floor_frac(ux)
            for ey in (0, 1):
                for ex in (0, 1):
                    cy, cx = int(yb0) + ey, int(xb0) + ex
                    wb = (fyb if ey else 1.0 - fyb) * (fxb if ex else 1.0 - fxb)
                    if not (0 <= cy < g.hb and 0 <= cx < g.wb) or wb == 0.0:
                        continue
                    view = views[cy * g.wb + cx]
                    for dy in (0, 1):
                        yy = y0 + dy
                        wy = fy if dy else 1.0 - fy
                        vy = (yy >= 0) & (yy < g.ha)
                        yc = np.clip(yy, 0, g.ha - 1)
                        for dx in (0, 1):
                            xx = x0 + dx
                            wx = fx if dx else 1.0 - fx
                            vx = (xx >= 0) & (xx < g.wa)
                            xc = np.clip(xx, 0, g.wa - 1)
                            if grid:
                                tap = view[yc[:, None], xc[None, :]]
                                tap = np.where(vy[:, None] & vx[None, :], tap, 0.0)
                                acc += wb * (wy[:, None] * wx[None, :]) * tap
                            else:
                                tap = np.where(vy & vx, view[yc, xc], 0.0)
                                acc += wb * (wy * wx) * tap
    return acc


def refocus_resampled(gamma_vm, g: Geometry, s: LensSampling, alphas) -> np.ndarray:
    """Refocused stack (n_alpha, out_h, out_w) in FP64 with the lens-plane
    coordinate taken on the sample grid ``s`` instead of detector B's pixel
    grid: the general form of the multilinear interpolation of Gamma
    (Section 4.1, refocusing optimisation), in which the interpolation points
    depend on the plane in all four coordinates.  With an integer grid
    (ox = oy = 0, sx = sy = 1, nx = Wb, ny = Hb) it is ``refocus``."""
    views = _views(gamma_vm, g)
    xr = np.arange(g.out_w, dtype=np.float64)
    yr = np.arange(g.out_h, dtype=np.float64)
    al = np.asarray(alphas, dtype=np.float64).reshape(-1)
    out = np.empty((al.size, g.out_h, g.out_w), dtype=np.float64)
    for k, a in enumerate(al):
        out[k] = _resampled_sum(views, g, s, a, xr, yr, grid=True)
    return out


def refocus_resampled_pixels(gamma_vm, g: Geometry, s: LensSampling, alphas, ys, xs):
    """``refocus_resampled`` at the listed output pixels: (n_alpha, len(ys))."""
    views = _views(gamma_vm, g)
    xr = np.asarray(xs, dtype=np.float64).reshape(-1)
    yr = np.asarray(ys, dtype=np.float64).reshape(-1)
    al = np.asarray(alphas, dtype=np.float64).reshape(-1)
    out = np.empty((al.size, xr.size), dtype=np.float64)
    for k, a in enumerate(al):
        out[k] = _resampled_sum(views, g, s, a, xr, yr, grid=False)
    return out
