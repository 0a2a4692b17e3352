"""Phantoms with a known refocusing answer (test inputs only).

* ``point_gamma``  -- a closed-form Gamma with no frames: every view rho_b holds
  the bilinear splat of one point placed where a plane alpha_star maps the
  output pixel rho_o in that view.  Refocusing at alpha_star must put the
  largest value exactly at rho_o.
* ``point_frames`` -- frames of a plenoptic point object: per frame, iid
  Exp(1) intensities L(rho_b) on detector B's lens-plane pixels; detector B
  counts Poisson(lam L); detector A counts Poisson(lam * sum_b L(rho_b)
  splat_b(rho_a)).  Then E[Gamma(rho_a, rho_b)] = lam^2 splat_b(rho_a), so the
  correlation function of these frames is a noisy copy of ``point_gamma``.
"""
import numpy as np


def _splat_1d(p, size):
    x0 = int(np.floor(p))
    f = p - x0
    w = np.zeros(size)
    if 0 <= x0 < size:
        w[x0] += 1.0 - f
    if 0 <= x0 + 1 < size:
        w[x0 + 1] += f
    return w, f


def point_position(g, alpha, xo, yo, xb, yb):
    px = alpha * (xo - g.ca_x) + g.ca_x + (1.0 - alpha) * g.mag_x * (xb - g.cb_x)
    py = alpha * (yo - g.ca_y) + g.ca_y + (1.0 - alpha) * g.mag_y * (yb - g.cb_y)
    return px, py


def point_gamma(g, alpha_star, xo, yo):
    """View-major Gamma (Pb, Pa) and the exact refocused value at (xo, yo)."""
    gam = np.zeros((g.hb * g.wb, g.ha * g.wa))
    peak = 0.0
    for yb in range(g.hb):
        for xb in range(g.wb):
            px, py = point_position(g, alpha_star, xo, yo, xb, yb)
            wx, fx = _splat_1d(px, g.wa)
            wy, fy = _splat_1d(py, g.ha)
            gam[yb * g.wb + xb] = np.outer(wy, wx).reshape(-1)
            peak += ((1 - fx) ** 2 + fx ** 2) * ((1 - fy) ** 2 + fy ** 2)
    return gam, peak


def point_frames(g, alpha_star, xo, yo, n, lam, seed):
    """(A counts (n, Pa), B counts (n, Pb)) as uint8 for the point object."""
    gam, _ = point_gamma(g, alpha_star, xo, yo)     # (Pb, Pa) splat weights
    rng = np.random.default_rng(seed)
    lens = rng.exponential(1.0, size=(n, g.hb * g.wb))
    b = rng.poisson(lam * lens)
    a = rng.poisson(lam * (lens @ gam))
    return np.minimum(a, 255).astype(np.uint8), np.minimum(b, 255).astype(np.uint8)
