"""Raw sensor frames with both detectors side by side, as the paper's
SwissSPAD2 files hold them (Section "Input Dataset"): each frame is frame_h
rows of frame_w 1-bit pixels, the left half imaging detector A and the right
half detector B, packed row-major 8 pixels per byte with the first pixel in
the least-significant bit, frames back to back with no header.

Only input files are produced here: given the two detectors' 0/1 images, the
region of interest they occupy inside each half, and filler pixels for the
rest of the frame.
"""
from __future__ import annotations

import os

import numpy as np


def compose_sidebyside(a, b, frame_w: int, frame_h: int, roi_x: int, roi_y: int,
                       rng: np.random.Generator | None = None, fill: float = 0.1) -> np.ndarray:
    """(n, roi_h, roi_w) 0/1 images of A and B -> (n, frame_h, frame_w) 0/1
    raw frames with A's region in the left half, B's in the right half, and
    random filler (probability `fill`) elsewhere."""
    a = np.asarray(a, dtype=np.uint8)
    b = np.asarray(b, dtype=np.uint8)
    n, rh, rw = a.shape
    if b.shape != a.shape or frame_w % 2 or roi_x + rw > frame_w // 2 or roi_y + rh > frame_h:
        raise ValueError("region does not fit the half frame")
    rng = rng or np.random.default_rng(0)
    raw = (rng.random((n, frame_h, frame_w)) < fill).astype(np.uint8)
    half = frame_w // 2
    raw[:, roi_y:roi_y + rh, roi_x:roi_x + rw] = a
    raw[:, roi_y:roi_y + rh, half + roi_x:half + roi_x + rw] = b
    return raw


def pack_raw_frames(raw) -> np.ndarray:
    """(n, frame_h, frame_w) 0/1 -> (n, ceil(frame_h*frame_w/8)) bytes."""
    raw = np.asarray(raw, dtype=np.uint8)
    return np.packbits(raw.reshape(raw.shape[0], -1), axis=1, bitorder="little")


def write_frame_files(directory: str, packed, frames_per_file) -> list[str]:
    """Writes packed raw frames to consecutive files; frames_per_file is an
    int or a list of counts.  Returns the paths in order."""
    packed = np.asarray(packed, dtype=np.uint8)
    counts = ([int(frames_per_file)] * ((packed.shape[0] + frames_per_file - 1) // frames_per_file)
              if np.isscalar(frames_per_file) else [int(c) for c in frames_per_file])
    paths, i = [], 0
    for k, c in enumerate(counts):
        c = min(c, packed.shape[0] - i)
        path = os.path.join(directory, f"frames_{k:05d}.bin")
        packed[i:i + c].tofile(path)
        paths.append(path)
        i += c
    if i != packed.shape[0]:
        raise ValueError("frame counts do not cover every frame")
    return paths
