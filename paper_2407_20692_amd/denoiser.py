"""Learned denoiser of refocused planes: binding of the ``cpi_denoiser_*``,
``cpi_image_quality`` and ``cpi_nn_*`` entry points of ``include/cpi.h``.

Argument marshalling only; the network runs in the library's kernels (BF16
matrix-core convolutions, FP32 master weights and Adam).  Device tensors come
from torch; bfloat16 tensors are passed as their raw 16-bit storage.
"""
from __future__ import annotations

import ctypes
import math
from ctypes import c_char, c_int32, c_int64, c_size_t, c_void_p

from .binding import _check, _dev_ptr, _stream, _torch, alloc_workspace, lib


class LayerInfo(ctypes.Structure):
    _fields_ = [
        ("name_raw", c_char * 16),
        ("cin", c_int32), ("cout", c_int32), ("ks", c_int32),
        ("cin_used", c_int32), ("cout_used", c_int32),
        ("weight_offset", c_int64), ("bias_offset", c_int64),
    ]

    @property
    def name(self) -> str:
        return self.name_raw.decode()

    @property
    def weight_count(self) -> int:
        return self.cout * self.ks * self.ks * self.cin


def layers():
    n = c_int32(0)
    _check(lib.cpi_denoiser_layer_count(ctypes.byref(n)))
    out = []
    for i in range(n.value):
        info = LayerInfo()
        _check(lib.cpi_denoiser_layer_info(i, ctypes.byref(info)))
        out.append(info)
    return out


def param_count() -> int:
    n = c_int64(0)
    _check(lib.cpi_denoiser_param_count(ctypes.byref(n)))
    return n.value


def workspace_size(batch: int, h: int, w: int, train: bool) -> int:
    out = c_size_t(0)
    _check(lib.cpi_denoiser_workspace_size(batch, h, w, 1 if train else 0, ctypes.byref(out)))
    return out.value


def init_params(seed: int, device="cuda"):
    """He-normal weights (fan-in of the used input channels), zero biases and
    zero weights for padded channels; drawn on the host from a seeded torch
    generator, then copied to the device."""
    torch = _torch()
    gen = torch.Generator()
    gen.manual_seed(seed)
    p = torch.zeros(param_count(), dtype=torch.float32)
    for L in layers():
        w = torch.zeros(L.cout, L.ks, L.ks, L.cin)
        std = math.sqrt(2.0 / (L.cin_used * L.ks * L.ks))
        w[:L.cout_used, :, :, :L.cin_used] = torch.randn(
            L.cout_used, L.ks, L.ks, L.cin_used, generator=gen) * std
        p[L.weight_offset:L.weight_offset + L.weight_count] = w.reshape(-1)
    return p.to(device)


def layer_view(params, L: LayerInfo):
    """(weights [cout, ks, ks, cin], biases [cout]) views of a parameter array."""
    w = params[L.weight_offset:L.weight_offset + L.weight_count].view(L.cout, L.ks, L.ks, L.cin)
    b = params[L.bias_offset:L.bias_offset + L.cout]
    return w, b


def _planes(t, what, batch, h, w):
    return _dev_ptr(t, what, dtype=_torch().float32, numel=batch * h * w)


class Denoiser:
    """Parameters, Adam state and workspaces of one denoiser on one device."""

    def __init__(self, seed: int = 0, device="cuda", params=None):
        torch = _torch()
        self.device = torch.device(device)
        self.params = init_params(seed, self.device) if params is None else params.to(
            self.device, torch.float32).contiguous()
        if self.params.numel() != param_count():
            raise ValueError("parameter array has the wrong size")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}
        self.loss = torch.zeros(4, dtype=torch.float32, device=self.device)

    def _workspace(self, batch, h, w, train):
        key = (batch, h, w, bool(train))
        if key not in self._ws:
            self._ws[key] = alloc_workspace(workspace_size(batch, h, w, train), self.device)
        return self._ws[key]

    def forward(self, planes, out=None, stream=None):
        """Denoised planes [batch, h, w] (FP32 device tensors)."""
        torch = _torch()
        b, h, w = planes.shape
        if out is None:
            out = torch.empty_like(planes)
        ws = self._workspace(b, h, w, False)
        _check(lib.cpi_denoiser_forward(
            _dev_ptr(self.params, "params", dtype=torch.float32), b, h, w,
            _planes(planes, "planes", b, h, w), _planes(out, "out", b, h, w),
            _dev_ptr(ws, "workspace"), ws.numel(), _stream(stream)))
        return out

    def train_step(self, planes, targets, lr: float = 1e-3, stream=None):
        """One Adam step; returns a device scalar holding the batch loss."""
        torch = _torch()
        b, h, w = planes.shape
        if tuple(targets.shape) != (b, h, w):
            raise ValueError("targets must match planes")
        ws = self._workspace(b, h, w, True)
        self.step += 1
        _check(lib.cpi_denoiser_train_step(
            _dev_ptr(self.params, "params", dtype=torch.float32),
            _dev_ptr(self.m, "adam_m", dtype=torch.float32),
            _dev_ptr(self.v, "adam_v", dtype=torch.float32),
            self.step, float(lr), b, h, w,
            _planes(planes, "planes", b, h, w), _planes(targets, "targets", b, h, w),
            _dev_ptr(self.loss, "loss"), _dev_ptr(ws, "workspace"), ws.numel(), _stream(stream)))
        return self.loss[0]

    def gradients(self, planes, targets, stream=None):
        """(loss, gradients) of one batch without an update."""
        torch = _torch()
        b, h, w = planes.shape
        ws = self._workspace(b, h, w, True)
        grads = torch.empty_like(self.params)
        loss = torch.zeros(4, dtype=torch.float32, device=self.device)
        _check(lib.cpi_denoiser_gradients(
            _dev_ptr(self.params, "params", dtype=torch.float32), b, h, w,
            _planes(planes, "planes", b, h, w), _planes(targets, "targets", b, h, w),
            _dev_ptr(loss, "loss"), _dev_ptr(grads, "grads"), _dev_ptr(ws, "workspace"),
            ws.numel(), _stream(stream)))
        return loss[0], grads

    def state(self):
        return {"params": self.params.detach().cpu(), "step": self.step}


def image_quality(pred, target, stream=None):
    """(psnr, ssim) per plane as FP64 device tensors."""
    torch = _torch()
    b, h, w = pred.shape
    if tuple(target.shape) != (b, h, w):
        raise ValueError("target must match pred")
    psnr = torch.empty(b, dtype=torch.float64, device=pred.device)
    ssim = torch.empty(b, dtype=torch.float64, device=pred.device)
    _check(lib.cpi_image_quality(_planes(pred, "pred", b, h, w), _planes(target, "target", b, h, w),
                                 b, h, w, _dev_ptr(psnr, "psnr"), _dev_ptr(ssim, "ssim"),
                                 _stream(stream)))
    return psnr, ssim


# ---- single kernels ------------------------------------------------------------------
def _bf(t, what, numel=None):
    return _dev_ptr(t, what, dtype=_torch().bfloat16, numel=numel)


def kpad(ks: int, c: int) -> int:
    return (ks * ks * c + 31) // 32 * 32


def pack_weights(w, transposed: bool = True, stream=None):
    """FP32 w [cout, ks, ks, cin] -> (w_packed [cout, kpad], w_packed_t [cin, kpad_t] or None)."""
    torch = _torch()
    cout, ks, _, cin = w.shape
    wf = torch.empty(cout, kpad(ks, cin), dtype=torch.bfloat16, device=w.device)
    wt = torch.empty(cin, kpad(ks, cout), dtype=torch.bfloat16, device=w.device) if transposed \
        else None
    _check(lib.cpi_nn_pack_weights(_dev_ptr(w, "w", dtype=torch.float32, numel=w.numel()),
                                   cout, cin, ks, _bf(wf, "w_packed"),
                                   _bf(wt, "w_packed_t") if wt is not None else None,
                                   _stream(stream)))
    return wf, wt


def conv2d(x, w_packed, ks: int, cout: int, bias=None, mask=None, relu=False, out=None,
           out_f32=None, stream=None):
    """x [b, h, w, cin] bfloat16, w_packed [cout, kpad] -> out (bfloat16) and/or out_f32."""
    torch = _torch()
    b, h, w, cin = x.shape
    n = b * h * w * cout
    if out is None and out_f32 is None:
        out = torch.empty(b, h, w, cout, dtype=torch.bfloat16, device=x.device)
    _check(lib.cpi_nn_conv2d(
        _bf(x, "x"), _bf(w_packed, "w_packed", cout * kpad(ks, cin)),
        _dev_ptr(bias, "bias", dtype=torch.float32, numel=cout) if bias is not None else None,
        _bf(mask, "mask", n) if mask is not None else None, 1 if relu else 0,
        b, h, w, cin, cout, ks, kpad(ks, cin),
        _bf(out, "out", n) if out is not None else None,
        _dev_ptr(out_f32, "out_f32", dtype=torch.float32, numel=n) if out_f32 is not None else None,
        _stream(stream)))
    return out if out is not None else out_f32


def conv2d_wgrad_workspace_size(b: int, h: int, w: int, cin: int, cout: int, ks: int) -> int:
    """Bytes of the partial-sum workspace conv2d_wgrad uses for this shape."""
    out = c_size_t(0)
    _check(lib.cpi_nn_conv2d_wgrad_workspace_size(b, h, w, cin, cout, ks, ctypes.byref(out)))
    return out.value


def conv2d_wgrad(x, dy, ks: int, dw, db=None, workspace=None, stream=None):
    """dw [cout, ks, ks, cin] FP32 += weight gradient (and db [cout] += bias
    gradient if given).  With a workspace (a uint8 device tensor of at least
    conv2d_wgrad_workspace_size bytes) the pixel splits are summed in a fixed
    order; without one they add with FP32 atomics."""
    torch = _torch()
    b, h, w, cin = x.shape
    cout = dy.shape[3]
    _check(lib.cpi_nn_conv2d_wgrad(_bf(x, "x"), _bf(dy, "dy", b * h * w * cout), b, h, w, cin,
                                   cout, ks,
                                   _dev_ptr(dw, "dw", dtype=torch.float32,
                                            numel=cout * ks * ks * cin),
                                   _dev_ptr(db, "db", dtype=torch.float32, numel=cout)
                                   if db is not None else None,
                                   _dev_ptr(workspace, "workspace") if workspace is not None
                                   else None,
                                   workspace.numel() * workspace.element_size()
                                   if workspace is not None else 0,
                                   _stream(stream)))
    return dw


def bias_grad(dy, db, stream=None):
    torch = _torch()
    c = dy.shape[-1]
    _check(lib.cpi_nn_bias_grad(_bf(dy, "dy"), dy.numel() // c, c,
                                _dev_ptr(db, "db", dtype=torch.float32, numel=c), _stream(stream)))
    return db


def maxpool2(x, stream=None):
    torch = _torch()
    b, h, w, c = x.shape
    out = torch.empty(b, h // 2, w // 2, c, dtype=torch.bfloat16, device=x.device)
    _check(lib.cpi_nn_maxpool2(_bf(x, "x"), b, h, w, c, _bf(out, "out"), _stream(stream)))
    return out


def maxpool2_grad(x, dout, stream=None):
    torch = _torch()
    b, h, w, c = x.shape
    dx = torch.empty_like(x)
    _check(lib.cpi_nn_maxpool2_grad(_bf(x, "x"), _bf(dout, "dout", dx.numel() // 4), b, h, w, c,
                                    _bf(dx, "dx"), _stream(stream)))
    return dx


def upsample2(x, stream=None):
    torch = _torch()
    b, h, w, c = x.shape
    out = torch.empty(b, 2 * h, 2 * w, c, dtype=torch.bfloat16, device=x.device)
    _check(lib.cpi_nn_upsample2(_bf(x, "x"), b, h, w, c, _bf(out, "out"), _stream(stream)))
    return out


def upsample2_grad(dout, mask=None, stream=None):
    torch = _torch()
    b, h2, w2, c = dout.shape
    dx = torch.empty(b, h2 // 2, w2 // 2, c, dtype=torch.bfloat16, device=dout.device)
    _check(lib.cpi_nn_upsample2_grad(_bf(dout, "dout"), b, h2 // 2, w2 // 2, c,
                                     _bf(mask, "mask", dx.numel()) if mask is not None else None,
                                     _bf(dx, "dx"), _stream(stream)))
    return dx


def concat(a, b, stream=None):
    torch = _torch()
    ca, cb = a.shape[-1], b.shape[-1]
    p = a.numel() // ca
    out = torch.empty(*a.shape[:-1], ca + cb, dtype=torch.bfloat16, device=a.device)
    _check(lib.cpi_nn_concat(_bf(a, "a"), _bf(b, "b", p * cb), p, ca, cb, _bf(out, "out"),
                             _stream(stream)))
    return out


def upsample2_concat(low, skip, stream=None):
    """[upsample2(low), skip] along channels."""
    torch = _torch()
    b, h, w, c1 = low.shape
    c2 = skip.shape[3]
    out = torch.empty(b, 2 * h, 2 * w, c1 + c2, dtype=torch.bfloat16, device=low.device)
    _check(lib.cpi_nn_upsample2_concat(_bf(low, "low"), _bf(skip, "skip", b * 4 * h * w * c2),
                                       b, h, w, c1, c2, _bf(out, "out"), _stream(stream)))
    return out


def upsample2_concat_grad(d, c1: int, mask=None, stream=None):
    """(dlow, dskip) of upsample2_concat for its output gradient d."""
    torch = _torch()
    b, h2, w2, c = d.shape
    dlow = torch.empty(b, h2 // 2, w2 // 2, c1, dtype=torch.bfloat16, device=d.device)
    dskip = torch.empty(b, h2, w2, c - c1, dtype=torch.bfloat16, device=d.device)
    _check(lib.cpi_nn_upsample2_concat_grad(_bf(d, "d"), b, h2 // 2, w2 // 2, c1, c - c1,
                                            _bf(mask, "mask", dlow.numel())
                                            if mask is not None else None,
                                            _bf(dlow, "dlow"), _bf(dskip, "dskip"),
                                            _stream(stream)))
    return dlow, dskip


def split(d, ca: int, stream=None):
    torch = _torch()
    c = d.shape[-1]
    p = d.numel() // c
    da = torch.empty(*d.shape[:-1], ca, dtype=torch.bfloat16, device=d.device)
    db = torch.empty(*d.shape[:-1], c - ca, dtype=torch.bfloat16, device=d.device)
    _check(lib.cpi_nn_split(_bf(d, "d"), p, ca, c - ca, _bf(da, "da"), _bf(db, "db"),
                            _stream(stream)))
    return da, db


def add_mask(x, add=None, mask=None, stream=None):
    n = x.numel()
    _check(lib.cpi_nn_add_mask(_bf(x, "x"), _bf(add, "add", n) if add is not None else None,
                               _bf(mask, "mask", n) if mask is not None else None, n,
                               _stream(stream)))
    return x


def mse(y, target, residual=None, stream=None):
    """(loss device scalar, dy bfloat16 [..., c]) for y [..., c] FP32."""
    torch = _torch()
    c = y.shape[-1]
    p = y.numel() // c
    loss = torch.zeros(4, dtype=torch.float32, device=y.device)
    dy = torch.empty(y.shape, dtype=torch.bfloat16, device=y.device)
    _check(lib.cpi_nn_mse(_dev_ptr(y, "y", dtype=torch.float32), c,
                          _dev_ptr(residual, "residual", dtype=torch.float32, numel=p)
                          if residual is not None else None,
                          _dev_ptr(target, "target", dtype=torch.float32, numel=p), p,
                          _dev_ptr(loss, "loss"), _bf(dy, "dy"), _stream(stream)))
    return loss[0], dy


def adam(w, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _torch()
    n = w.numel()
    f = torch.float32
    _check(lib.cpi_nn_adam(_dev_ptr(w, "w", dtype=f), _dev_ptr(g, "g", dtype=f, numel=n),
                           _dev_ptr(m, "m", dtype=f, numel=n), _dev_ptr(v, "v", dtype=f, numel=n),
                           n, step, lr, beta1, beta2, eps, _stream(stream)))
    return w
