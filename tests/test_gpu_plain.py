"""GPU check of the plain FP32 correlator against its a-priori error bound.

With exact FP32 sums (all integers below 2^24), the plain path rounds five
times (three divisions, one product, one subtraction), so per entry
    |gamma_f32 - Gamma| <= 5 * 2^-24 * (S_ab/N + (S_a/N)(S_b/N)) + 2^-48.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, generate_frames, pack_bits_lsb
from tests.gpu_util import dev, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def _plain(cpi, fa, fb, n, pa, pb, fmt, layout):
    import torch

    out = torch.full((pa * pb,), np.nan, dtype=torch.float32, device=dev())
    cpi.correlate_f32_plain(to_dev(fa), to_dev(fb), n, pa, pb, fmt, out, layout)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _bound(a, b, n):
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    sab = a64.T @ b64
    ma, mb = a64.mean(0), b64.mean(0)
    return 5 * 2.0 ** -24 * (sab / n + np.outer(ma, mb)) + 2.0 ** -48


@pytest.mark.parametrize("layout", [0, 1])
def test_tiny_workload_within_bound(cpi, layout):
    w = WORKLOADS["da32_db16_n1000_u8counts"]
    a, b = generate_frames(w, workers=1)
    log(f"case plain {w.name} layout={layout}")
    got = _plain(cpi, a, b, w.n_frames, w.pa, w.pb, cpi.FRAMES_U8, layout)
    ref = oracle.correlation(a, b, w.n_frames, w.pa, w.pb, oracle.FRAMES_U8)
    err = np.abs(got.astype(np.float64) - oracle.to_layout(ref["gamma"], layout).reshape(-1))
    bound = oracle.to_layout(_bound(a, b, w.n_frames), layout).reshape(-1)
    assert (err <= bound).all(), np.max(err / bound)


@pytest.mark.parametrize("n,pa,pb", [(777, 1000, 77), (20, 129, 300)])
def test_ragged_bits_within_bound(cpi, n, pa, pb):
    rng = np.random.default_rng(n + pa)
    a = (rng.random((n, pa)) < 0.3).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.3).astype(np.uint8)
    log(f"case plain bits n={n} pa={pa} pb={pb}")
    fa = np.concatenate([pack_bits_lsb(a).reshape(-1), np.zeros(16, np.uint8)])
    fb = np.concatenate([pack_bits_lsb(b).reshape(-1), np.zeros(16, np.uint8)])
    got = _plain(cpi, fa, fb, n, pa, pb, cpi.FRAMES_BIT1, 0)
    ref = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    err = np.abs(got.astype(np.float64) - ref["gamma"].T.reshape(-1))
    assert (err <= _bound(a, b, n).T.reshape(-1)).all()
