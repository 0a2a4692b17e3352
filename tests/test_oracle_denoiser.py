"""Pins of the denoiser oracle (CPU only).

Each oracle function is tied to something other than itself: brute-force
loops over the definition, a library routine (SciPy's 2-D correlation,
PyTorch's bfloat16 conversion), adjoint identities between a linear map and
its gradient, central finite differences of the whole network's loss, and
closed forms (Adam's first step, PSNR of a constant offset, SSIM of constant
planes).
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle.denoiser as dn


def _brute_conv(x, w, b):
    B, H, W, Cin = x.shape
    Cout, ks, _, _ = w.shape
    h = (ks - 1) // 2
    y = np.zeros((B, H, W, Cout))
    for n in range(B):
        for yy in range(H):
            for xx in range(W):
                for co in range(Cout):
                    s = b[co]
                    for ky in range(ks):
                        for kx in range(ks):
                            sy, sx = yy + ky - h, xx + kx - h
                            if 0 <= sy < H and 0 <= sx < W:
                                for ci in range(Cin):
                                    s += w[co, ky, kx, ci] * x[n, sy, sx, ci]
                    y[n, yy, xx, co] = s
    return y


@pytest.mark.parametrize("ks", [1, 3])
def test_conv_brute_force(ks):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 3))
    w = rng.standard_normal((4, ks, ks, 3))
    b = rng.standard_normal(4)
    assert np.allclose(dn.conv2d(x, w, b), _brute_conv(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv_single_channel_is_scipy_correlation():
    rng = np.random.default_rng(2)
    img = rng.standard_normal((9, 7))
    k = rng.standard_normal((3, 3))
    ref = scipy.signal.correlate2d(img, k, mode="same", boundary="fill")
    got = dn.conv2d(img[None, :, :, None], k[None, :, :, None])[0, :, :, 0]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_conv_delta_kernels():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 6, 6, 2))
    w = np.zeros((2, 3, 3, 2))
    w[0, 1, 1, 0] = w[1, 1, 1, 1] = 1.0          # centre tap: identity
    assert np.array_equal(dn.conv2d(x, w), x)
    w = np.zeros((1, 3, 3, 2))
    w[0, 1, 2, 1] = 1.0                          # right neighbour of channel 1
    y = dn.conv2d(x, w)[0, :, :, 0]
    assert np.array_equal(y[:, :5], x[0, :, 1:, 1])
    assert np.array_equal(y[:, 5], np.zeros(6))


@pytest.mark.parametrize("ks", [1, 3])
def test_conv_gradients_are_adjoints(ks):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 4, 3))
    w = rng.standard_normal((5, ks, ks, 3))
    dy = rng.standard_normal((2, 6, 4, 5))
    dx = rng.standard_normal((2, 6, 4, 3))
    dw = rng.standard_normal((5, ks, ks, 3))
    # <conv(x, w), dy> = <x, grad_input(dy, w)> = <w, grad_weight(x, dy)>
    lhs = np.sum(dn.conv2d(x, w) * dy)
    assert np.isclose(lhs, np.sum(x * dn.conv2d_grad_input(dy, w)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(w * dn.conv2d_grad_weight(x, dy, ks)), rtol=1e-12)
    # directional derivatives (exact for a bilinear map)
    assert np.isclose(np.sum((dn.conv2d(x + dx, w) - dn.conv2d(x, w)) * dy),
                      np.sum(dx * dn.conv2d_grad_input(dy, w)), rtol=1e-10)
    assert np.isclose(np.sum((dn.conv2d(x, w + dw) - dn.conv2d(x, w)) * dy),
                      np.sum(dw * dn.conv2d_grad_weight(x, dy, ks)), rtol=1e-10)
    assert np.allclose(dn.bias_grad(dy), dy.sum(axis=(0, 1, 2)))


def test_maxpool_brute_force_and_tie_rule():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 4, 6, 3))
    y = dn.maxpool2(x)
    for n in range(2):
        for i in range(2):
            for j in range(3):
                for c in range(3):
                    assert y[n, i, j, c] == max(x[n, 2 * i + a, 2 * j + b, c]
                                                for a in (0, 1) for b in (0, 1))
    # gradient = directional derivative where the maximum is unique
    d = rng.standard_normal(x.shape) * 1e-7
    g = rng.standard_normal(y.shape)
    assert np.isclose(np.sum((dn.maxpool2(x + d) - y) * g),
                      np.sum(d * dn.maxpool2_grad(x, g)), rtol=1e-6)
    # ties: the first position in window order (0,0), (0,1), (1,0), (1,1)
    t = np.array([[1.0, 2.0], [2.0, 2.0]]).reshape(1, 2, 2, 1)
    gt = dn.maxpool2_grad(t, np.array([[[[5.0]]]]))[0, :, :, 0]
    assert np.array_equal(gt, [[0.0, 5.0], [0.0, 0.0]])


def test_upsample_adjoint():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 3, 4, 5))
    u = dn.upsample2(x)
    assert u.shape == (2, 6, 8, 5)
    assert u[1, 5, 7, 4] == x[1, 2, 3, 4] and u[0, 2, 1, 0] == x[0, 1, 0, 0]
    g = rng.standard_normal(u.shape)
    assert np.isclose(np.sum(u * g), np.sum(x * dn.upsample2_grad(g)), rtol=1e-12)


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.01171875, -3.0e38, 1e-30]])
    v32 = v.astype(np.float32)
    ref = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(dn.round_bf16(v32.astype(np.float64)), ref)
    # ties to even: 1 + 2^-8 lies between 1 and 1 + 2^-7
    assert dn.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert dn.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_mse_and_adam_closed_forms():
    p = np.array([1.0, 2.0, 4.0])
    t = np.array([0.0, 2.0, 1.0])
    assert dn.mse(p, t) == (1.0 + 0.0 + 9.0) / 3.0
    assert np.array_equal(dn.mse_grad(p, t), 2.0 * (p - t) / 3.0)
    # first step from zero moments: m_hat = g, v_hat = g^2
    w = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -2.0, 0.0])
    w1, m, v = dn.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-8)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-16)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    for step in range(2, 6):
        w2, m, v = dn.adam_step(w1, g, m, v, step, lr=0.01, eps=1e-8)
        assert np.allclose(w1 - w2, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16)
        w1 = w2


def test_normalize_planes():
    rng = np.random.default_rng(8)
    p = rng.standard_normal((3, 8, 8)) * 5 + 2
    p[2] = 7.0
    x, mu, sd = dn.normalize_planes(p)
    assert np.allclose(x[:2].mean(axis=(1, 2)), 0, atol=1e-12)
    assert np.allclose(x[:2].std(axis=(1, 2)), 1, atol=1e-12)
    assert sd[2] == 1.0 and np.all(x[2] == 0.0)


def test_network_gradients_finite_differences():
    """Backward of the FP64 network against central differences of its loss."""
    rng = np.random.default_rng(9)
    params = dn.init_params(rng)
    for k in params:
        params[k] = (params[k][0], rng.standard_normal(params[k][1].shape) * 0.05)
    planes = rng.standard_normal((2, 8, 8))
    targets = planes * 0.5 + rng.standard_normal((2, 8, 8)) * 0.1
    loss, grads, _ = dn.loss_and_grads(params, planes, targets, bf16=False)
    assert loss > 0
    checks = 0
    for name in ("enc1a", "enc2b", "mid_b", "dec3a", "dec1a", "out"):
        w, b = params[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            h = 1e-5
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            fp = dn.loss_and_grads({**params, name: (wp, b)}, planes, targets, bf16=False)[0]
            fm = dn.loss_and_grads({**params, name: (wm, b)}, planes, targets, bf16=False)[0]
            fd = (fp - fm) / (2 * h)
            an = grads[name][0][idx]
            assert abs(fd - an) <= 1e-5 * max(1e-3, abs(fd)) + 1e-9, (name, idx, fd, an)
            checks += 1
        j = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[j] += 1e-5
        bm[j] -= 1e-5
        fd = (dn.loss_and_grads({**params, name: (w, bp)}, planes, targets, bf16=False)[0] -
              dn.loss_and_grads({**params, name: (w, bm)}, planes, targets, bf16=False)[0]) / 2e-5
        assert abs(fd - grads[name][1][j]) <= 1e-5 * max(1e-3, abs(fd)) + 1e-9
    assert checks == 18


def test_psnr_closed_form():
    rng = np.random.default_rng(10)
    t = rng.random((16, 16)) * 3.0
    rng_t = t.max() - t.min()
    for c in (0.1, 0.01):
        assert math.isclose(dn.psnr(t + c, t), 10 * math.log10(rng_t ** 2 / c ** 2), rel_tol=1e-12)
    assert dn.psnr(t, t) == math.inf


def test_ssim_closed_forms():
    rng = np.random.default_rng(11)
    t = rng.random((16, 16))
    assert math.isclose(dn.ssim(t, t), 1.0, rel_tol=1e-12)
    # constant target (range taken as 1) and constant prediction a above it:
    # every window has zero variances, so SSIM = C1 / (a^2 + C1)
    tc = np.full((12, 12), 3.0)
    for a in (0.0, 0.02, 0.5):
        assert math.isclose(dn.ssim(tc + a, tc), 0.01 ** 2 / (a * a + 0.01 ** 2), rel_tol=1e-12)
    # more noise, lower SSIM
    s = [dn.ssim(t + rng.standard_normal(t.shape) * e, t) for e in (0.01, 0.1, 0.5)]
    assert s[0] > s[1] > s[2]
    w = dn.gaussian_window()
    assert w.shape == (11, 11) and math.isclose(w.sum(), 1.0) and w[5, 5] == w.max()


def _ramp_ssim_closed_form(w, a, c, sigma, k1, k2, size=11):
    """SSIM of pred = a*t + c against the ramp t(y, x) = x / (w - 1).

    The target's range is 1 and its minimum 0, so both planes keep their
    values.  Inside every window the target has mean m = x_c / (w - 1) (x_c the
    window's centre column: the weights are symmetric) and variance
    v = sum_r g(r) r^2 / ((w - 1)^2 sum_r g(r)) with g(r) = exp(-r^2 / (2 sigma^2))
    over r = -(size-1)/2 .. (size-1)/2 (the window is separable and its row
    factor sums to 1); the prediction has mean a*m + c, variance a^2 v and
    covariance a v with the target."""
    h = (size - 1) // 2
    g = [math.exp(-(r * r) / (2.0 * sigma * sigma)) for r in range(-h, h + 1)]
    v = sum(gi * r * r for gi, r in zip(g, range(-h, h + 1))) / (sum(g) * (w - 1) ** 2)
    c1, c2 = k1 * k1, k2 * k2
    vals = []
    for x0 in range(w - size + 1):
        mb = (x0 + h) / (w - 1)
        ma = a * mb + c
        vals.append((2 * ma * mb + c1) * (2 * a * v + c2) /
                    ((ma * ma + mb * mb + c1) * (a * a * v + v + c2)))
    return sum(vals) / len(vals)


def test_ssim_ramp_closed_form_fixes_window_and_constants():
    """The Gaussian window's sigma (1.5) and the constants K1 = 0.01, K2 = 0.03
    of the SSIM reading enter a hand-computable value on a linear ramp."""
    w, hgt = 24, 13
    t = np.tile(np.arange(w, dtype=np.float64) / (w - 1), (hgt, 1))
    for a, c in ((0.5, 0.1), (0.8, -0.05), (1.7, 0.3)):
        pred = a * t + c
        want = _ramp_ssim_closed_form(w, a, c, 1.5, 0.01, 0.03)
        assert math.isclose(dn.ssim(pred, t), want, rel_tol=1e-10), (a, c)
        # the closed form separates the readings: another sigma or K2 moves
        # the value far beyond the tolerance above
        for sig, k2 in ((1.0, 0.03), (1.5, 0.01), (2.0, 0.03)):
            other = _ramp_ssim_closed_form(w, a, c, sig, 0.01, k2)
            assert abs(other - want) > 1e-4, (a, c, sig, k2)
            assert math.isclose(dn.ssim(pred, t, sigma=sig, k2=k2), other, rel_tol=1e-10)
    # an offset-only prediction leaves the contrast term at 1
    pred = t + 0.2
    want = _ramp_ssim_closed_form(w, 1.0, 0.2, 1.5, 0.01, 0.03)
    assert math.isclose(dn.ssim(pred, t), want, rel_tol=1e-10)
