"""Chaotic-light speckle frames for two detectors (synthetic, seeded).

Physical model (a stand-in for the paper's SwissSPAD2 acquisitions):

* field      E = g_sigma (*) (X + iY) on the Da grid, X, Y iid N(0, 1), the
               convolution done by FFT on a grid padded by ``PAD`` pixels and
               then cropped; sigma = 0.85 px gives a speckle grain of ~2 px
               (intensity autocorrelation FWHM = 2.355 sigma).
* intensity  I = |E|^2 / E|E|^2, so I ~ Exp(1) per pixel.
* detector A sees I * T (T a binary transmission mask); detector B sees the
  M x M block mean of I (M = Wa / Wb), unmasked.
* counts     Poisson(mean_counts * I * T) on A and Poisson(mean_counts * Ibar)
             on B, clipped to uint8 ("poisson_u8");
  or clicks  Bernoulli(1 - exp(-lam * I * T)) and likewise on B
             ("binary_u8" as bytes 0/1, "binary_packed" as 1 bit per pixel).

Frames are generated in blocks of ``BLOCK`` frames; block k draws from the k-th
child of ``SeedSequence(seed)``, so any frame range is reproducible on its own
and a streamed run sees exactly the frames of a single-shot run.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import scipy.fft as sfft

from .workloads import Workload, workload_seed, mask_seed

SIGMA = 0.85
PAD = 8
BLOCK = 1000


def chunk_seed_sequences(seed: int, n_blocks: int):
    return np.random.SeedSequence(seed).spawn(n_blocks)


def slit_mask(wa: int, ha: int, seed: int, n_slits: int = 3) -> np.ndarray:
    """Binary mask with ``n_slits`` vertical slits (1 = transmitting).

    Slit widths are 2..6 px per 128 px of detector width, the slits are
    0.6*Ha long and vertically centred, their left edges lie in the central
    80% of the width and consecutive slits are separated by at least their
    width.
    """
    rng = np.random.default_rng(seed)
    scale = wa / 128.0
    lo_w = max(1, int(round(2 * scale)))
    hi_w = max(lo_w, int(round(6 * scale)))
    x_lo = int(np.floor(0.1 * wa))
    x_hi = int(np.ceil(0.9 * wa))
    length = max(1, int(round(0.6 * ha)))
    y0 = (ha - length) // 2
    for _attempt in range(1000):
        widths = rng.integers(lo_w, hi_w + 1, size=n_slits)
        lefts = np.sort(rng.integers(x_lo, x_hi, size=n_slits))
        ok = True
        for s in range(n_slits):
            if lefts[s] + widths[s] > x_hi:
                ok = False
            if s > 0 and lefts[s] - (lefts[s - 1] + widths[s - 1]) < widths[s - 1]:
                ok = False
        if ok:
            break
    else:  # pragma: no cover - the search space is large for every workload
        raise RuntimeError("could not place slits")
    mask = np.zeros((ha, wa), dtype=np.uint8)
    for s in range(n_slits):
        mask[y0:y0 + length, lefts[s]:lefts[s] + widths[s]] = 1
    return mask


def _gaussian_transfer(hp: int, wp: int, sigma: float) -> np.ndarray:
    ky = np.fft.fftfreq(hp)[:, None]
    kx = np.fft.fftfreq(wp)[None, :]
    return np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx * kx + ky * ky))


def speckle_block(w: Workload, mask: np.ndarray, seq: np.random.SeedSequence,
                  n: int) -> tuple[np.ndarray, np.ndarray]:
    """``n`` frame pairs as uint8 arrays of shape (n, Pa) and (n, Pb).

    Values are counts (``poisson_u8``) or 0/1 (binary encodings).
    """
    rng = np.random.default_rng(seq)
    hp, wp = w.ha + 2 * PAD, w.wa + 2 * PAD
    gt = _gaussian_transfer(hp, wp, SIGMA)
    gt32 = gt.astype(np.float32)
    # E|E|^2 = 2 * sum(g^2) for unit-variance real and imaginary noise;
    # Parseval on the padded grid gives sum(g^2) = mean(|G|^2).
    mean_int = 2.0 * float(np.mean(gt * gt))
    m = w.wa // w.wb
    out_a = np.empty((n, w.pa), dtype=np.uint8)
    out_b = np.empty((n, w.pb), dtype=np.uint8)
    step = 250
    for s in range(0, n, step):
        k = min(step, n - s)
        noise = np.empty((k, hp, wp), dtype=np.complex64)
        noise.real = rng.standard_normal((k, hp, wp), dtype=np.float32)
        noise.imag = rng.standard_normal((k, hp, wp), dtype=np.float32)
        field = sfft.ifft2(sfft.fft2(noise, axes=(1, 2)) * gt32, axes=(1, 2))
        inten = (field.real ** 2 + field.imag ** 2)[:, PAD:PAD + w.ha, PAD:PAD + w.wa]
        inten /= mean_int
        ia = inten * mask[None, :, :]
        ib = inten.reshape(k, w.hb, m, w.wb, m).mean(axis=(2, 4))
        if w.encoding == "poisson_u8":
            ca = rng.poisson(w.mean_counts * ia)
            cb = rng.poisson(w.mean_counts * ib)
            out_a[s:s + k] = np.minimum(ca, 255).reshape(k, -1)
            out_b[s:s + k] = np.minimum(cb, 255).reshape(k, -1)
        else:
            ua = rng.random(ia.shape, dtype=np.float32)
            ub = rng.random(ib.shape, dtype=np.float32)
            out_a[s:s + k] = (ua < -np.expm1(-w.lam * ia)).reshape(k, -1)
            out_b[s:s + k] = (ub < -np.expm1(-w.lam * ib)).reshape(k, -1)
    return out_a, out_b


def _block_job(args):
    w, mask, seq, n = args
    return speckle_block(w, mask, seq, n)


def generate_frames(w: Workload, start: int = 0, count: int | None = None,
                    workers: int | None = None, seed: int | None = None
                    ) -> tuple[np.ndarray, np.ndarray]:
    """Frames [start, start+count) of workload ``w`` as 0/1 or count bytes.

    ``start`` must be a multiple of ``BLOCK``.  Blocks are generated in
    parallel with up to ``workers`` processes (default: host cores, at most 16).
    """
    if count is None:
        count = w.n_frames - start
    if start % BLOCK:
        raise ValueError("start must be a multiple of the block size")
    seed = workload_seed(w) if seed is None else seed
    mask = slit_mask(w.wa, w.ha, mask_seed(w))
    first = start // BLOCK
    last = (start + count + BLOCK - 1) // BLOCK
    seqs = chunk_seed_sequences(seed, max(last, 1))
    jobs = []
    for b in range(first, last):
        n_b = min(BLOCK, start + count - b * BLOCK)
        jobs.append((w, mask, seqs[b], n_b))
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)))
    workers = max(1, min(workers, len(jobs)))
    if workers == 1:
        parts = [_block_job(j) for j in jobs]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(_block_job, jobs))
    a = np.concatenate([p[0] for p in parts], axis=0)
    b = np.concatenate([p[1] for p in parts], axis=0)
    return a, b


def pack_bits_lsb(frames: np.ndarray) -> np.ndarray:
    """Pack 0/1 frames (n, P) into (n, ceil(P/8)) bytes, pixel 8j+k in bit k of byte j."""
    frames = np.ascontiguousarray(frames, dtype=np.uint8)
    return np.packbits(frames, axis=1, bitorder="little")
