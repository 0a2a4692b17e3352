"""Seeded synthetic inputs for correlation plenoptic imaging.

This package produces frames only: chaotic-light speckle images on the two
detectors, binary transmission masks, photon counting / SPAD binarisation, bit
packing and the refocus-plane grids.  It holds none of the arithmetic of the
correlation function or of refocusing, so both the CPU oracle and the HIP path
can take their inputs from here without sharing any of the method's code.
"""
from .workloads import WORKLOADS, Workload, alphas_for, workload_seed, mask_seed
from .speckle import (
    slit_mask,
    speckle_block,
    generate_frames,
    pack_bits_lsb,
    chunk_seed_sequences,
)
from .rawframes import compose_sidebyside, pack_raw_frames, write_frame_files

__all__ = [
    "WORKLOADS",
    "Workload",
    "alphas_for",
    "workload_seed",
    "mask_seed",
    "slit_mask",
    "speckle_block",
    "generate_frames",
    "pack_bits_lsb",
    "chunk_seed_sequences",
    "compose_sidebyside",
    "pack_raw_frames",
    "write_frame_files",
]
