"""The learned denoiser inside the imaging pipeline.

Training pairs come from the method itself: for one stream of frames, the
planes refocused after its first ``n_few`` frames are the inputs and the same
planes (same alphas) after its first ``n_full`` frames are the targets, so
every run yields one pair per refocus plane.  The plain pipeline is both the
judge of the denoiser (PSNR / SSIM against its full-stream planes) and its
fallback: the denoiser is used only where it beats the plain pipeline given
the same wall time, i.e. where the denoised ``n_few``-frame planes are better
than the plain planes from the ``n_eq`` frames the plain pipeline processes
in the time of ``n_few`` frames plus inference.

Every step of the computation runs in the library's kernels (correlation,
refocusing, the network, the quality measures); torch holds device memory
and streams and assembles batches by index (plain copies).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from .binding import FRAMES_BIT1, Stream, _torch, alloc_workspace, refocus_workspace_size
from .denoiser import Denoiser, image_quality


def _plane_shape(geom):
    return geom.out_h, geom.out_w


def prefix_planes(frames_a, frames_b, pa: int, pb: int, geom, alphas, counts, outs,
                  chunk: int = 10000):
    """Refocuses one stream after its first counts[0] < counts[1] < ... frames.

    frames_a, frames_b: device uint8 tensors of packed 1-bit frames (frame-major).
    outs[i]: contiguous FP32 device tensor of len(alphas) planes for counts[i].
    """
    st = Stream(pa, pb, FRAMES_BIT1, chunk)
    ws = alloc_workspace(refocus_workspace_size(geom, len(alphas)), frames_a.device)
    pos = 0
    try:
        for n, out in zip(counts, outs):
            if n < pos:
                raise ValueError("counts must be ascending")
            while pos < n:
                k = min(chunk, n - pos)
                st.push(frames_a[pos:pos + k], frames_b[pos:pos + k], k)
                pos += k
            st.refocus(geom, alphas, out, workspace=ws)
    finally:
        st.close()
    return outs


def make_pairs(frame_source, alpha_source, runs: int, pa: int, pb: int, geom, n_few: int,
               n_full: int, chunk: int = 10000, log=None):
    """(inputs, targets): FP32 device tensors [runs * n_alpha, h, w].

    frame_source(r) -> (frames_a, frames_b) device tensors of at least n_full
    frames for run r; alpha_source(r) -> the run's refocus parameters.
    """
    torch = _torch()
    h, w = _plane_shape(geom)
    inputs = targets = None
    for r in range(runs):
        fa, fb = frame_source(r)
        al = alpha_source(r)
        na = len(al)
        if inputs is None:
            inputs = torch.empty(runs * na, h, w, dtype=torch.float32, device=fa.device)
            targets = torch.empty_like(inputs)
        prefix_planes(fa, fb, pa, pb, geom, al, [n_few, n_full],
                      [inputs[r * na:(r + 1) * na], targets[r * na:(r + 1) * na]], chunk)
        if log and (r + 1) % max(1, runs // 10) == 0:
            log(f"pairs: run {r + 1}/{runs}")
        del fa, fb
    return inputs, targets


def train(net: Denoiser, inputs, targets, epochs: int, batch: int = 16, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Adam over shuffled batches; returns the mean training loss per epoch."""
    torch = _torch()
    n, h, w = inputs.shape
    nb = n // batch
    if nb < 1:
        raise ValueError("fewer pairs than one batch")
    gen = torch.Generator()
    gen.manual_seed(seed)
    xb = torch.empty(batch, h, w, dtype=torch.float32, device=inputs.device)
    tb = torch.empty_like(xb)
    history = []
    for e in range(epochs):
        perm = torch.randperm(n, generator=gen).to(inputs.device)
        total = torch.zeros((), dtype=torch.float32, device=inputs.device)
        for i in range(nb):
            idx = perm[i * batch:(i + 1) * batch]
            torch.index_select(inputs, 0, idx, out=xb)
            torch.index_select(targets, 0, idx, out=tb)
            total += net.train_step(xb, tb, lr)
        history.append(float(total) / nb)
        if log:
            log(f"epoch {e + 1}/{epochs}: loss {history[-1]:.5f}")
    return history


def denoise_batched(net: Denoiser, planes, batch: int = 32, out=None):
    """Denoised planes, in batches of at most `batch` planes."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(planes)
    for i in range(0, planes.shape[0], batch):
        net.forward(planes[i:i + batch], out=out[i:i + batch])
    return out


def quality(pred, target):
    """Mean PSNR and SSIM over planes, and the per-plane values (host lists)."""
    psnr, ssim = image_quality(pred, target)
    p, s = psnr.cpu().tolist(), ssim.cpu().tolist()
    return sum(p) / len(p), sum(s) / len(s), p, s


@dataclass
class Policy:
    """Outcome of the comparison at equal wall time."""
    use_denoiser: bool
    n_few: int
    n_eq: int
    psnr_denoised: float
    psnr_plain_eq: float
    ssim_denoised: float
    ssim_plain_eq: float
    reason: str = ""
    extra: dict = field(default_factory=dict)


def decide(psnr_den, ssim_den, psnr_eq, ssim_eq, n_few, n_eq) -> Policy:
    """The denoiser is used only if it beats the plain pipeline at equal wall
    time on both PSNR and SSIM (validation planes); otherwise the plain
    pipeline runs on n_eq frames."""
    use = psnr_den > psnr_eq and ssim_den > ssim_eq
    why = ("denoised planes better than plain planes at equal time" if use else
           "plain pipeline at equal time is at least as good: fall back to it")
    return Policy(use, n_few, n_eq, psnr_den, psnr_eq, ssim_den, ssim_eq, why)


def apply(net: Denoiser | None, policy: Policy | None, planes_few, planes_plain=None):
    """Planes delivered by the pipeline: denoised few-frame planes when the
    policy selects the denoiser (planes whose output is not finite fall back
    to their plain input), else the plain planes (``planes_plain``, or the
    few-frame planes when none are given)."""
    torch = _torch()
    if net is None or policy is None or not policy.use_denoiser:
        return planes_plain if planes_plain is not None else planes_few
    out = denoise_batched(net, planes_few)
    bad = ~torch.isfinite(out).flatten(1).all(dim=1)
    if bool(bad.any()):
        out[bad] = planes_few[bad]
    return out


def fit_linear(ns, ts):
    """Least-squares t = a + b * n."""
    m = len(ns)
    sx, sy = sum(ns), sum(ts)
    sxx = sum(x * x for x in ns)
    sxy = sum(x * y for x, y in zip(ns, ts))
    b = (m * sxy - sx * sy) / (m * sxx - sx * sx)
    return (sy - b * sx) / m, b


def equal_time_frames(t_budget_ms: float, a_ms: float, b_ms_per_frame: float, n_min: int,
                      n_max: int) -> int:
    if b_ms_per_frame <= 0:
        return n_max
    n = int(math.floor((t_budget_ms - a_ms) / b_ms_per_frame))
    return max(n_min, min(n_max, n))
