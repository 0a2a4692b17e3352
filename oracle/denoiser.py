"""Oracle of the learned denoiser (test infrastructure only).

The paper has no denoiser; this module writes out, in FP64 NumPy, the model
the library trains on the planes its own pipeline produces: refocused planes
from few frames mapped to the same planes from many frames.  The model is a
convolutional encoder-decoder (U-Net form), read as follows:

* normalisation: each input plane p is shifted and scaled by its own mean and
  population standard deviation (sigma = 1 for a constant plane):
  x = (p - mu) / sigma;
* network f: four levels of widths 32, 64, 128, 256.  Each encoder level is
  two 3x3 convolutions with zero padding, each followed by ReLU; levels are
  joined by 2x2 max-pooling.  Each decoder level upsamples by 2 (nearest),
  concatenates [upsampled, encoder output of that level] along channels and
  applies two 3x3 convolutions with ReLU.  A final 1x1 convolution (no ReLU)
  gives one channel;
* output: (x + f(x)) * sigma + mu;
* loss: mean squared error, over all pixels of the batch, between x + f(x)
  and the target plane normalised with the input's (mu, sigma);
* optimiser: Adam with bias-corrected moments on FP32 master weights.

Convolutions are cross-correlations: y[p, co] = b[co] + sum over taps
(ky, kx) and input channels ci of w[co, ky, kx, ci] * x[p + (ky - h, kx - h), ci]
with h = (ks - 1) / 2 and x = 0 outside the image.  Max-pooling passes the
gradient to the first window position holding the maximum, in the order
(0,0), (0,1), (1,0), (1,1).

Storage precision.  The library stores activations, gradients of activations
and the weights fed to the matrix cores as bfloat16, and sums in FP32.  With
``bf16=True`` the network functions here round every such stored value to
the nearest bfloat16 (ties to even) at the same points, so that the library
and the oracle compute the same function up to the order of their sums.

Image quality (evaluation of the denoiser):
* PSNR with the data range of the target plane, max(t) - min(t);
* SSIM with an 11 x 11 Gaussian window (sigma 1.5, truncated, normalised to
  sum 1) over every position where the window fits inside the plane,
  K1 = 0.01, K2 = 0.03, both planes mapped to [0, 1] by the target's
  minimum and range.

Pinned by ``tests/test_oracle_denoiser.py`` (brute force, library routines,
finite differences, adjoint identities and closed forms).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

WIDTHS = (32, 64, 128, 256)


# ---- bfloat16 -----------------------------------------------------------------
def round_bf16(x):
    """Nearest bfloat16 value of every element (ties to even), as float64.

    bfloat16 keeps 8 significant bits: with x = m * 2^e, 0.5 <= |m| < 1, the
    result is round_half_even(m * 2^8) * 2^(e - 8).  Values are assumed to lie
    in the normal range of bfloat16 (or be zero).
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0), e - 8)


def _maybe(x, bf16):
    return round_bf16(x) if bf16 else x


# ---- layers (NHWC, float64) ---------------------------------------------------
def shift(x, dy, dx):
    """s[b, y, x, c] = x[b, y + dy, x + dx, c], zero where that is outside."""
    b, h, w, c = x.shape
    out = np.zeros_like(x)
    ys0, ys1 = max(0, -dy), min(h, h - dy)
    xs0, xs1 = max(0, -dx), min(w, w - dx)
    if ys0 < ys1 and xs0 < xs1:
        out[:, ys0:ys1, xs0:xs1, :] = x[:, ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx, :]
    return out


def conv2d(x, w, bias=None):
    """x [B, H, W, Cin], w [Cout, ks, ks, Cin] -> [B, H, W, Cout]."""
    cout, ks, _, cin = w.shape
    h = (ks - 1) // 2
    y = np.zeros(x.shape[:3] + (cout,), dtype=np.float64)
    for ky in range(ks):
        for kx in range(ks):
            y += shift(x, ky - h, kx - h) @ w[:, ky, kx, :].T
    if bias is not None:
        y += bias
    return y


def conv2d_grad_input(dy, w):
    """Gradient of sum(conv2d(x, w) * dy) with respect to x."""
    cout, ks, _, cin = w.shape
    h = (ks - 1) // 2
    dx = np.zeros(dy.shape[:3] + (cin,), dtype=np.float64)
    for ky in range(ks):
        for kx in range(ks):
            dx += shift(dy, -(ky - h), -(kx - h)) @ w[:, ky, kx, :]
    return dx


def conv2d_grad_weight(x, dy, ks):
    """Gradient of sum(conv2d(x, w) * dy) with respect to w [Cout, ks, ks, Cin]."""
    h = (ks - 1) // 2
    cin, cout = x.shape[3], dy.shape[3]
    dw = np.zeros((cout, ks, ks, cin), dtype=np.float64)
    for ky in range(ks):
        for kx in range(ks):
            xs = shift(x, ky - h, kx - h)
            dw[:, ky, kx, :] = dy.reshape(-1, cout).T @ xs.reshape(-1, cin)
    return dw


def bias_grad(dy):
    return dy.reshape(-1, dy.shape[3]).sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    b, h, w, c = x.shape
    return x.reshape(b, h // 2, 2, w // 2, 2, c).max(axis=(2, 4))


def maxpool2_grad(x, dout):
    """Gradient of the 2x2 max to the first maximal position of each window."""
    b, h, w, c = x.shape
    win = x.reshape(b, h // 2, 2, w // 2, 2, c).transpose(0, 1, 3, 5, 2, 4).reshape(
        b, h // 2, w // 2, c, 4)
    first = np.argmax(win, axis=4)          # argmax returns the first maximum
    onehot = (np.arange(4) == first[..., None]) * dout[..., None]
    return onehot.reshape(b, h // 2, w // 2, c, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(
        b, h, w, c)


def upsample2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def upsample2_grad(dout):
    b, h2, w2, c = dout.shape
    return dout.reshape(b, h2 // 2, 2, w2 // 2, 2, c).sum(axis=(2, 4))


def mse(pred, target):
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d))


def mse_grad(pred, target):
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return 2.0 * d / d.size


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def normalize_planes(p):
    """p [B, H, W] -> (x, mu [B], sigma [B]) with x = (p - mu) / sigma."""
    p = np.asarray(p, np.float64)
    mu = p.mean(axis=(1, 2))
    var = ((p - mu[:, None, None]) ** 2).mean(axis=(1, 2))
    sd = np.where(var > 0, np.sqrt(var), 1.0)
    return (p - mu[:, None, None]) / sd[:, None, None], mu, sd


# ---- the network ----------------------------------------------------------------
@dataclass(frozen=True)
class Layer:
    name: str
    cin: int
    cout: int
    ks: int


def layers():
    """Convolutions in execution order, at their logical channel counts."""
    w1, w2, w3, w4 = WIDTHS
    return [
        Layer("enc1a", 1, w1, 3), Layer("enc1b", w1, w1, 3),
        Layer("enc2a", w1, w2, 3), Layer("enc2b", w2, w2, 3),
        Layer("enc3a", w2, w3, 3), Layer("enc3b", w3, w3, 3),
        Layer("mid_a", w3, w4, 3), Layer("mid_b", w4, w4, 3),
        Layer("dec3a", w4 + w3, w3, 3), Layer("dec3b", w3, w3, 3),
        Layer("dec2a", w3 + w2, w2, 3), Layer("dec2b", w2, w2, 3),
        Layer("dec1a", w2 + w1, w1, 3), Layer("dec1b", w1, w1, 3),
        Layer("out", w1, 1, 1),
    ]


def init_params(rng):
    """He-normal weights and zero biases, {name: (w [Cout, ks, ks, Cin], b)}."""
    p = {}
    for L in layers():
        std = math.sqrt(2.0 / (L.cin * L.ks * L.ks))
        p[L.name] = (rng.standard_normal((L.cout, L.ks, L.ks, L.cin)) * std, np.zeros(L.cout))
    return p


def forward(params, x, bf16=True):
    """x [B, H, W] normalised planes -> (x + f(x) [B, H, W], cache).

    H and W must be multiples of 8.
    """
    q = lambda a: _maybe(a, bf16)
    c = {"x": q(x[..., None])}
    W = {k: (q(w), b) for k, (w, b) in params.items()}

    def conv(name, inp, act=True):
        w, b = W[name]
        y = conv2d(inp, w, b)
        return q(relu(y)) if act else y

    h = c["x"]
    skips = []
    for lvl, (a, bname) in enumerate([("enc1a", "enc1b"), ("enc2a", "enc2b"), ("enc3a", "enc3b")]):
        c[a] = conv(a, h)
        c[bname] = conv(bname, c[a])
        skips.append(bname)
        c[f"pool{lvl + 1}"] = maxpool2(c[bname])
        h = c[f"pool{lvl + 1}"]
    c["mid_a"] = conv("mid_a", h)
    c["mid_b"] = conv("mid_b", c["mid_a"])
    h = c["mid_b"]
    for lvl, (a, bname) in zip((3, 2, 1), [("dec3a", "dec3b"), ("dec2a", "dec2b"),
                                           ("dec1a", "dec1b")]):
        c[f"cat{lvl}"] = np.concatenate([upsample2(h), c[skips[lvl - 1]]], axis=3)
        c[a] = conv(a, c[f"cat{lvl}"])
        c[bname] = conv(bname, c[a])
        h = c[bname]
    c["out"] = conv("out", h, act=False)            # FP32 in the library: not rounded
    y = np.asarray(x, np.float64) + c["out"][..., 0]
    return y, c


def backward(params, cache, dy, bf16=True):
    """Gradients {name: (dw, db)} of sum(y * dy) for the forward pass `cache`.

    dy [B, H, W] is the gradient of the loss with respect to the output
    x + f(x); it is stored (rounded) before the first convolution uses it.
    """
    q = lambda a: _maybe(a, bf16)
    c = cache
    W = {k: q(w) for k, (w, _b) in params.items()}
    grads = {}

    def back(name, inp, g, mask_act=None):
        """Weight and bias gradients of layer `name`, and the input gradient
        (masked by the ReLU of the layer that produced `inp`, if given)."""
        grads[name] = (conv2d_grad_weight(inp, g, W[name].shape[1]), bias_grad(g))
        gi = conv2d_grad_input(g, W[name])
        if mask_act is not None:
            gi = gi * (mask_act > 0)
        return q(gi)

    g = q(dy[..., None])
    g = back("out", c["dec1b"], g, c["dec1b"])
    skip_grad = {}
    for lvl, (a, bname), below in zip((1, 2, 3), [("dec1a", "dec1b"), ("dec2a", "dec2b"),
                                                  ("dec3a", "dec3b")],
                                      ("dec2b", "dec3b", "mid_b")):
        g = back(bname, c[a], g, c[a])
        gcat = back(a, c[f"cat{lvl}"], g)
        cu = c[below].shape[3]
        gup, skip_grad[lvl] = gcat[..., :cu], gcat[..., cu:]
        g = q(upsample2_grad(gup) * (c[below] > 0))
    g = back("mid_b", c["mid_a"], g, c["mid_a"])
    g = back("mid_a", c["pool3"], g)
    for lvl, (a, bname) in zip((3, 2, 1), [("enc3a", "enc3b"), ("enc2a", "enc2b"),
                                           ("enc1a", "enc1b")]):
        g = q((maxpool2_grad(c[bname], g) + skip_grad[lvl]) * (c[bname] > 0))
        g = back(bname, c[a], g, c[a])
        if a == "enc1a":
            grads[a] = (conv2d_grad_weight(c["x"], g, 3), bias_grad(g))
        else:
            prev = {"enc3a": "pool2", "enc2a": "pool1"}[a]
            g = back(a, c[prev], g)
    return grads


def loss_and_grads(params, planes, targets, bf16=True):
    """Loss of one batch (planes and targets [B, H, W], raw) and its gradients."""
    x, mu, sd = normalize_planes(planes)
    t = (np.asarray(targets, np.float64) - mu[:, None, None]) / sd[:, None, None]
    y, cache = forward(params, x, bf16)
    return mse(y, t), backward(params, cache, mse_grad(y, t), bf16), y


def denoise(params, planes, bf16=True):
    x, mu, sd = normalize_planes(planes)
    y, _ = forward(params, x, bf16)
    return y * sd[:, None, None] + mu[:, None, None]


# ---- image quality ------------------------------------------------------------------
def psnr(pred, target):
    t = np.asarray(target, np.float64)
    rng = float(t.max() - t.min())
    err = mse(pred, t)
    if err == 0.0:
        return math.inf
    return 10.0 * math.log10(rng * rng / err)


def gaussian_window(size=11, sigma=1.5):
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(r * r) / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def ssim(pred, target, size=11, sigma=1.5, k1=0.01, k2=0.03):
    t = np.asarray(target, np.float64)
    lo = float(t.min())
    rng = float(t.max() - lo)
    if rng == 0.0:
        rng = 1.0
    a = (np.asarray(pred, np.float64) - lo) / rng
    b = (t - lo) / rng
    c1, c2 = (k1 * 1.0) ** 2, (k2 * 1.0) ** 2
    w = gaussian_window(size, sigma)
    h, wd = a.shape
    vals = []
    for y in range(h - size + 1):
        for x in range(wd - size + 1):
            pa = a[y:y + size, x:x + size]
            pb = b[y:y + size, x:x + size]
            ma, mb = (w * pa).sum(), (w * pb).sum()
            va = (w * (pa - ma) ** 2).sum()
            vb = (w * (pb - mb) ** 2).sum()
            cab = (w * (pa - ma) * (pb - mb)).sum()
            vals.append(((2 * ma * mb + c1) * (2 * cab + c2)) /
                        ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    return float(np.mean(vals))
