"""Device-side generation of the same chaotic-light frames (large workloads).

The physical model is the one of ``synth.speckle`` (Gaussian-filtered complex
noise, Exp(1) intensity, a slit mask on detector A, M x M binning on detector
B, SPAD clicks with P = 1 - exp(-lam * I)); random numbers come from a seeded
torch generator on the device, so frames are reproducible for a given seed and
device but differ from the NumPy generator's.  Only inputs are produced here:
the frames are then handed to both the oracle and the library unchanged.
"""
from __future__ import annotations

import numpy as np

from .speckle import PAD, SIGMA, slit_mask
from .workloads import Workload, mask_seed, workload_seed


def _transfer(torch, hp, wp, dev):
    ky = torch.fft.fftfreq(hp, device=dev, dtype=torch.float64)[:, None]
    kx = torch.fft.fftfreq(wp, device=dev, dtype=torch.float64)[None, :]
    return torch.exp(-2.0 * (np.pi * SIGMA) ** 2 * (kx * kx + ky * ky)).to(torch.float32)


def pack_bits_lsb_torch(x):
    """(n, P) 0/1 uint8 -> (n, ceil(P/8)) bytes, pixel 8j+k in bit k of byte j."""
    import torch

    n, p = x.shape
    pad = (-p) % 8
    if pad:
        x = torch.cat([x, torch.zeros(n, pad, dtype=x.dtype, device=x.device)], dim=1)
    w = (1 << torch.arange(8, device=x.device, dtype=torch.int32)).view(1, 1, 8)
    return (x.view(n, -1, 8).to(torch.int32) * w).sum(dim=2).to(torch.uint8)


def generate_binary_frames_gpu(w: Workload, count: int | None = None, seed: int | None = None,
                               device="cuda", chunk: int = 2000, mask_seed_value: int | None = None):
    """Binary frames (clicks) of workload ``w`` on the device, packed 8 per byte.

    ``mask_seed_value`` replaces the workload's slit-mask seed (a different
    object per run).

    Returns (frames_a, frames_b) as uint8 device tensors of shape
    (count, ceil(Pa/8)) and (count, ceil(Pb/8)).
    """
    import torch

    count = w.n_frames if count is None else count
    seed = workload_seed(w) if seed is None else seed
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    ms = mask_seed(w) if mask_seed_value is None else mask_seed_value
    mask = torch.from_numpy(slit_mask(w.wa, w.ha, ms)).to(dev, torch.float32)
    hp, wp = w.ha + 2 * PAD, w.wa + 2 * PAD
    gt = _transfer(torch, hp, wp, dev)
    mean_int = 2.0 * float((gt.double() ** 2).mean())
    m = w.wa // w.wb
    out_a = torch.empty((count, (w.pa + 7) // 8), dtype=torch.uint8, device=dev)
    out_b = torch.empty((count, (w.pb + 7) // 8), dtype=torch.uint8, device=dev)
    for s in range(0, count, chunk):
        k = min(chunk, count - s)
        re = torch.randn((k, hp, wp), generator=gen, device=dev)
        im = torch.randn((k, hp, wp), generator=gen, device=dev)
        field = torch.fft.ifft2(torch.fft.fft2(torch.complex(re, im)) * gt)
        inten = (field.real ** 2 + field.imag ** 2)[:, PAD:PAD + w.ha, PAD:PAD + w.wa] / mean_int
        ia = inten * mask
        ib = inten.reshape(k, w.hb, m, w.wb, m).mean(dim=(2, 4))
        ua = torch.rand(ia.shape, generator=gen, device=dev)
        ub = torch.rand(ib.shape, generator=gen, device=dev)
        ca = (ua < -torch.expm1(-w.lam * ia)).to(torch.uint8).reshape(k, -1)
        cb = (ub < -torch.expm1(-w.lam * ib)).to(torch.uint8).reshape(k, -1)
        out_a[s:s + k] = pack_bits_lsb_torch(ca)
        out_b[s:s + k] = pack_bits_lsb_torch(cb)
    return out_a, out_b
