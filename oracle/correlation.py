"""Oracle for the correlation function Gamma (test infrastructure only).

Definition followed: Eq. (1) of the paper (Section "CPI algorithm", item 1),

    Gamma[j,k,m,n] = (1/N) sum_i A^i[j,m] B^i[k,n]
                     - ((1/N) sum_i A^i[j,m]) ((1/N) sum_i B^i[k,n]),

with both terms normalised by the total frame count N (not N-1).  Writing
rho_a for the pixel (j, m) of detector A and rho_b for the pixel (k, n) of
detector B, and S_a, S_b, S_ab for the per-pixel sums and the sum of products,

    Gamma[rho_a, rho_b] = (N * S_ab - S_a * S_b) / N^2            (exactly).

The paper evaluates the sum of products "by matrix multiplication" (Section
4.1, cross-correlation optimisation); so does this oracle: S_ab = A^T B is one
float64 matrix product, which is exact because every product and every partial
sum is an integer below 2^53 (checked before use), so no summation order can
round.  The numerator is then formed in int64 and divided once in IEEE FP64:

    gamma = float64(numer) / float64(N * N).

That is the correctly rounded value of numer / N^2 whenever |numer| < 2^53.

Frame encodings (the paper's data are 1-bit frames, Section "Input Dataset"):
  * FRAMES_U8:   one byte per pixel, frame-major, pixel index y*W + x;
  * FRAMES_BIT1: 8 pixels per byte, pixel 8j+k in bit k of byte j (LSB
                 first), every frame padded to a whole number of bytes.
"""
from __future__ import annotations

import numpy as np

FRAMES_U8 = 0
FRAMES_BIT1 = 1

GAMMA_VIEW_MAJOR = 0   # Gamma stored [rho_b][rho_a]: Pb views of Ha x Wa
GAMMA_PIXEL_MAJOR = 1  # Gamma stored [rho_a][rho_b]

_TWO53 = 2 ** 53
_TWO63 = 2 ** 63


def frame_bytes(npix: int, fmt: int) -> int:
    return npix if fmt == FRAMES_U8 else (npix + 7) // 8


def unpack_frames(frames, n: int, npix: int, fmt: int) -> np.ndarray:
    """Frames as an (n, npix) uint8 array of pixel values."""
    raw = np.ascontiguousarray(np.asarray(frames, dtype=np.uint8)).reshape(-1)
    fb = frame_bytes(npix, fmt)
    if raw.size < n * fb:
        raise ValueError("frame buffer too small")
    raw = raw[: n * fb].reshape(n, fb)
    if fmt == FRAMES_U8:
        return raw
    if fmt == FRAMES_BIT1:
        bits = np.unpackbits(raw, axis=1, bitorder="little")
        return np.ascontiguousarray(bits[:, :npix])
    raise ValueError("unknown frame format")


def overflow_ok(n: int, amax: int, bmax: int) -> bool:
    """True when every integer in the exact evaluation fits int64 and N^2 < 2^53."""
    return n * n * max(amax, 1) * max(bmax, 1) < _TWO63 and n * n < _TWO53


def _exact_products(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """S_ab[p, q] = sum_i a[i, p] * b[i, q] as exact int64.

    One float64 matrix product: exact because N * max|a| * max|b| < 2^53,
    which the int64 bound checked by the caller implies for every N.
    """
    n = a.shape[0]
    amax = int(a.max(initial=0))
    bmax = int(b.max(initial=0))
    if n * amax * bmax >= _TWO53:
        raise OverflowError("sum of products not exact in float64")
    s = a.T.astype(np.float64) @ b.astype(np.float64)
    return s.astype(np.int64)


def correlation(frames_a, frames_b, n: int, pa: int, pb: int, fmt: int,
                rows_a=None, cols_b=None) -> dict:
    """Exact Gamma for n frame pairs, pixel-major ([rho_a][rho_b]).

    ``rows_a`` / ``cols_b`` (index arrays) restrict the output to a subset of
    A pixels / B pixels; the per-pixel sums are returned for the subset.

    Returns a dict with ``numer`` (int64), ``sum_a``, ``sum_b`` (int64),
    ``gamma`` (float64) and ``gamma_f32`` (float32 rounding of ``gamma``).
    """
    if n <= 0 or pa <= 0 or pb <= 0:
        raise ValueError("n, pa and pb must be positive")
    a = unpack_frames(frames_a, n, pa, fmt)
    b = unpack_frames(frames_b, n, pb, fmt)
    if rows_a is not None:
        a = a[:, np.asarray(rows_a)]
    if cols_b is not None:
        b = b[:, np.asarray(cols_b)]
    amax = int(a.max(initial=0))
    bmax = int(b.max(initial=0))
    if not overflow_ok(n, amax, bmax):
        raise OverflowError("N^2 * max|a| * max|b| must stay below 2^63 and N^2 below 2^53")
    sum_a = a.sum(axis=0, dtype=np.int64)
    sum_b = b.sum(axis=0, dtype=np.int64)
    s_ab = _exact_products(a, b)
    numer = np.int64(n) * s_ab - np.outer(sum_a, sum_b)
    gamma = numer.astype(np.float64) / np.float64(n * n)
    return {
        "numer": numer,
        "sum_a": sum_a,
        "sum_b": sum_b,
        "gamma": gamma,
        "gamma_f32": gamma.astype(np.float32),
    }


def to_layout(pixel_major: np.ndarray, layout: int) -> np.ndarray:
    """Re-express a [rho_a][rho_b] array in the requested storage layout."""
    if layout == GAMMA_PIXEL_MAJOR:
        return np.ascontiguousarray(pixel_major)
    if layout == GAMMA_VIEW_MAJOR:
        return np.ascontiguousarray(pixel_major.T)
    raise ValueError("unknown layout")
