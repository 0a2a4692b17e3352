"""Workload shapes for the synthetic stand-ins of the paper's SwissSPAD2 data.

The paper measures on 1-bit frames of two 256x256 regions of interest (Section
"Input Dataset"; benchmarks in Section 4.2 at 128x128 and 256x256).  That data
set is not public, so seeded speckle frames of the same format and sizes stand
in for it.  Each workload is named by its detector sizes, frame count and
frame encoding.
"""
from dataclasses import dataclass

import numpy as np

SEED_BASE = 2_0692_000


@dataclass(frozen=True)
class Workload:
    name: str
    index: int          # position in the list of workloads; fixes the seeds
    wa: int             # detector A (spatial detector Da) width, px
    ha: int             # detector A height, px
    wb: int             # detector B (lens-plane detector Db) width, px
    hb: int             # detector B height, px
    n_frames: int       # N, number of frame pairs
    encoding: str       # "poisson_u8" | "binary_u8" | "binary_packed"
    n_alpha: int        # refocus planes
    alpha_lo: float = 0.5
    alpha_hi: float = 1.5
    chunk: int = 0      # frames per streamed chunk (0: single shot)
    mean_counts: float = 0.5     # Poisson mean per transmitting pixel
    lam: float = 1.0 / 9.0       # SPAD exposure: P(click) = 1 - exp(-lam * I)

    @property
    def pa(self) -> int:
        return self.wa * self.ha

    @property
    def pb(self) -> int:
        return self.wb * self.hb

    @property
    def binary(self) -> bool:
        return self.encoding != "poisson_u8"


WORKLOADS = {
    w.name: w
    for w in [
        Workload("da32_db16_n1000_u8counts", 0, 32, 32, 16, 16, 1000,
                 "poisson_u8", 5),
        Workload("da128_db64_n20000_u8bin", 1, 128, 128, 64, 64, 20000,
                 "binary_u8", 32),
        Workload("da256_db128_n100000_bit1", 2, 256, 256, 128, 128, 100000,
                 "binary_packed", 128),
        Workload("da128_db64_stream200x1000_bit1", 3, 128, 128, 64, 64,
                 200000, "binary_packed", 32, chunk=1000),
        # the paper's benchmark configuration: 256 x 256 regions on both
        # detectors, 11 files of 512 frames, 261 refocus planes (Section 4.2)
        Workload("da256_db256_files11_bit1", 4, 256, 256, 256, 256, 11 * 512,
                 "binary_packed", 261),
        # learned denoiser: planes from the first 500 frames of a stream mapped
        # to the same planes from its first 50000 frames, 32 planes per run with
        # alphas drawn in [0.5, 1.5] and a different slit mask per run
        Workload("da128_db64_denoise500to50000_bit1", 5, 128, 128, 64, 64, 50000,
                 "binary_packed", 32),
    ]
}


def workload_seed(w: Workload) -> int:
    return SEED_BASE + w.index


def mask_seed(w: Workload) -> int:
    return SEED_BASE + w.index + 100


def alphas_for(w: Workload) -> np.ndarray:
    """Refocus-plane parameters: n_alpha values evenly spaced, endpoints kept."""
    return np.linspace(w.alpha_lo, w.alpha_hi, w.n_alpha)
