"""GPU parity of the exact correlator (cpi_correlate) against the CPU oracle.

Gamma (FP64), its FP32 rounding, the int64 numerator and the per-pixel sums
must be bit-identical to the oracle's.  Sizes span several work-group tiles
and ragged tails; the full-size case runs the bench configuration and is
checked on sampled views plus exact integer identities over every entry.
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth import WORKLOADS, generate_frames, pack_bits_lsb
from tests.gpu_util import assert_bit_exact, dev, log, oracle_in_layout, run_correlate, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAYOUTS = [oracle.GAMMA_VIEW_MAJOR, oracle.GAMMA_PIXEL_MAJOR]


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


@pytest.mark.parametrize("name", ["gamma_u8_3frames.json", "gamma_bit1_4frames.json",
                                  "gamma_u8_large_values.json"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_hand_worked_examples(cpi, name, layout):
    with open(os.path.join(GOLDEN, name)) as f:
        fx = json.load(f)
    fmt = cpi.FRAMES_U8 if fx["fmt"] == "u8" else cpi.FRAMES_BIT1
    fa = np.frombuffer(bytes.fromhex("".join(fx["frames_a_hex"])), dtype=np.uint8)
    fb = np.frombuffer(bytes.fromhex("".join(fx["frames_b_hex"])), dtype=np.uint8)
    # device buffers must be 16-byte aligned and hold whole frames; pad the tail
    fa = np.concatenate([fa, np.zeros(16, np.uint8)])
    fb = np.concatenate([fb, np.zeros(16, np.uint8)])
    log(f"case {name} layout={layout}")
    got = run_correlate(cpi, fa, fb, fx["n"], fx["pa"], fx["pb"], fmt, layout)
    ref = oracle.correlation(fa, fb, fx["n"], fx["pa"], fx["pb"], fmt)
    assert_bit_exact(got, oracle_in_layout(ref, layout))
    assert got["numer"].reshape(-1).tolist() == oracle.to_layout(
        np.array(fx["numer"]), layout).reshape(-1).tolist()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_tiny_workload_u8_counts(cpi, layout):
    w = WORKLOADS["da32_db16_n1000_u8counts"]
    a, b = generate_frames(w, workers=1)
    log(f"case {w.name} layout={layout}")
    ref = oracle.correlation(a, b, w.n_frames, w.pa, w.pb, oracle.FRAMES_U8)
    got = run_correlate(cpi, a, b, w.n_frames, w.pa, w.pb, cpi.FRAMES_U8, layout)
    assert_bit_exact(got, oracle_in_layout(ref, layout))
    again = run_correlate(cpi, a, b, w.n_frames, w.pa, w.pb, cpi.FRAMES_U8, layout)
    assert_bit_exact(again, got, "rerun ")


CASES = [
    # (n, pa, pb, kind)
    (1, 40, 24, "u8"),
    (2, 300, 17, "bits"),
    (777, 1000, 77, "u8"),
    (777, 1000, 77, "u8_binary"),
    (777, 1001, 77, "bits"),
    (513, 257, 255, "bits"),
    (2049, 600, 300, "u8_large"),
    (1536, 512, 512, "bits"),
    (64, 129, 1, "u8_large"),
]


@pytest.mark.parametrize("n,pa,pb,kind", CASES)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_ragged_shapes(cpi, n, pa, pb, kind, layout):
    rng = np.random.default_rng(n * 31 + pa * 7 + pb)
    if kind == "u8":
        a = rng.integers(0, 100, size=(n, pa), dtype=np.uint8)
        b = rng.integers(0, 100, size=(n, pb), dtype=np.uint8)
    elif kind == "u8_large":
        a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
        b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
    else:
        a = (rng.random((n, pa)) < 0.3).astype(np.uint8)
        b = (rng.random((n, pb)) < 0.3).astype(np.uint8)
    fmt = cpi.FRAMES_BIT1 if kind == "bits" else cpi.FRAMES_U8
    fa = pack_bits_lsb(a) if kind == "bits" else a
    fb = pack_bits_lsb(b) if kind == "bits" else b
    # frame buffers padded to a 16-byte multiple (the ABI requires aligned starts)
    fa = np.concatenate([fa.reshape(-1), np.zeros(16, np.uint8)])
    fb = np.concatenate([fb.reshape(-1), np.zeros(16, np.uint8)])
    log(f"case n={n} pa={pa} pb={pb} kind={kind} layout={layout}")
    ref = oracle.correlation(fa, fb, n, pa, pb, fmt)
    got = run_correlate(cpi, fa, fb, n, pa, pb, fmt, layout)
    assert_bit_exact(got, oracle_in_layout(ref, layout))


def test_binary_bytes_match_packed_bits(cpi):
    rng = np.random.default_rng(5)
    n, pa, pb = 3000, 700, 130
    a = (rng.random((n, pa)) < 0.1).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.1).astype(np.uint8)
    log("case u8 0/1 vs packed bits")
    g1 = run_correlate(cpi, a, b, n, pa, pb, cpi.FRAMES_U8, cpi.GAMMA_VIEW_MAJOR)
    g2 = run_correlate(cpi, np.concatenate([pack_bits_lsb(a).reshape(-1), np.zeros(16, np.uint8)]),
                       np.concatenate([pack_bits_lsb(b).reshape(-1), np.zeros(16, np.uint8)]),
                       n, pa, pb, cpi.FRAMES_BIT1, cpi.GAMMA_VIEW_MAJOR)
    assert_bit_exact(g1, g2)


@pytest.mark.parametrize("enc", ["auto", "int8"])
@pytest.mark.parametrize("n,pa,pb,kind", [(777, 1001, 77, "bits"), (1536, 512, 512, "bits"),
                                          (4099, 300, 260, "u8_binary"), (1, 33, 18, "bits"),
                                          (5000, 2048, 640, "bits")])
def test_binary_encodings(cpi, enc, n, pa, pb, kind):
    """Binary frames through either matrix-core encoding (FP4 with FP32 sums,
    int8 with int32 sums) give the oracle's results bit for bit; every frame
    of one column pair set, so a sum reaches n."""
    rng = np.random.default_rng(n + pa)
    a = (rng.random((n, pa)) < 0.2).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.2).astype(np.uint8)
    a[:, pa - 1] = 1
    b[:, 0] = 1
    fmt = cpi.FRAMES_BIT1 if kind == "bits" else cpi.FRAMES_U8
    fa = pack_bits_lsb(a) if kind == "bits" else a
    fb = pack_bits_lsb(b) if kind == "bits" else b
    fa = np.concatenate([fa.reshape(-1), np.zeros(16, np.uint8)])
    fb = np.concatenate([fb.reshape(-1), np.zeros(16, np.uint8)])
    log(f"case encoding={enc} n={n} pa={pa} pb={pb} kind={kind}")
    ref = oracle.correlation(fa, fb, n, pa, pb, fmt)
    before = cpi.get_mma_encoding()
    cpi.set_mma_encoding(cpi.MMA_INT8 if enc == "int8" else cpi.MMA_AUTO)
    try:
        got = run_correlate(cpi, fa, fb, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR)
    finally:
        cpi.set_mma_encoding(before)
    assert_bit_exact(got, oracle_in_layout(ref, cpi.GAMMA_VIEW_MAJOR))


def test_frames_past_one_ingest_pass(cpi):
    """2^24 + 4099 bit frames, more than one ingest pass takes: folded in
    blocks through the running sums, under either matrix-core encoding;
    every output bit-exact against the oracle."""
    n = (1 << 24) + 4099
    pa, pb = 40, 24
    rng = np.random.default_rng(24)
    fa = rng.integers(0, 256, size=(n, (pa + 7) // 8), dtype=np.uint8)
    fb = rng.integers(0, 256, size=(n, (pb + 7) // 8), dtype=np.uint8)
    fa = np.concatenate([fa.reshape(-1), np.zeros(16, np.uint8)])
    fb = np.concatenate([fb.reshape(-1), np.zeros(16, np.uint8)])
    ref = oracle.correlation(fa, fb, n, pa, pb, oracle.FRAMES_BIT1)
    before = cpi.get_mma_encoding()
    try:
        for enc in (cpi.MMA_AUTO, cpi.MMA_INT8):
            log(f"case frames past one ingest pass n={n} pa={pa} pb={pb} encoding={enc}")
            cpi.set_mma_encoding(enc)
            got = run_correlate(cpi, fa, fb, n, pa, pb, cpi.FRAMES_BIT1, cpi.GAMMA_VIEW_MAJOR)
            assert_bit_exact(got, oracle_in_layout(ref, cpi.GAMMA_VIEW_MAJOR))
    finally:
        cpi.set_mma_encoding(before)


@pytest.mark.parametrize("n", [131008, 131073, 270000])
def test_int32_flush_passes(cpi, n):
    """Byte frames beyond 131008 frames fold int32 partial sums into int64."""
    rng = np.random.default_rng(n)
    pa, pb = 96, 40
    a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
    b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
    a[:, 0] = 255
    b[:, 0] = 255     # worst-case products in one column pair
    log(f"case multipass n={n}")
    ref = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    got = run_correlate(cpi, a, b, n, pa, pb, cpi.FRAMES_U8, cpi.GAMMA_VIEW_MAJOR)
    assert_bit_exact(got, oracle_in_layout(ref, cpi.GAMMA_VIEW_MAJOR))


def test_paper_like_full_size(cpi):
    """Da 128x128, Db 64x64, N = 20000 binary bytes, in the bench configuration.
    Checked: 64 sampled views against the oracle element by element, every row
    and column sum of the numerator against its O(N(Pa+Pb)) integer identity,
    Freivalds products, the per-pixel sums, and a bitwise-identical rerun."""
    import torch

    w = WORKLOADS["da128_db64_n20000_u8bin"]
    a, b = generate_frames(w)
    n, pa, pb = w.n_frames, w.pa, w.pb
    log(f"case {w.name} full size")
    got = run_correlate(cpi, a, b, n, pa, pb, cpi.FRAMES_U8, cpi.GAMMA_VIEW_MAJOR)
    num = got["numer"].reshape(pb, pa)          # view-major
    rng = np.random.default_rng(77)
    views = np.sort(rng.choice(pb, size=64, replace=False))
    ref = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8, cols_b=views)
    assert np.array_equal(num[views], ref["numer"].T)
    assert np.array_equal(got["gamma"].reshape(pb, pa)[views], ref["gamma"].T)
    assert np.array_equal(got["gamma_f32"].reshape(pb, pa)[views], ref["gamma_f32"].T)
    a64 = a.astype(np.int64)
    b64 = b.astype(np.int64)
    sa, sb = a64.sum(axis=0), b64.sum(axis=0)
    assert np.array_equal(got["sum_a"], sa) and np.array_equal(got["sum_b"], sb)
    ta, tb = a64.sum(axis=1), b64.sum(axis=1)
    rows_a = n * (a64 * tb[:, None]).sum(axis=0) - sa * sb.sum()   # sum over rho_b
    rows_b = n * (b64 * ta[:, None]).sum(axis=0) - sb * sa.sum()   # sum over rho_a
    assert np.array_equal(num.sum(axis=0), rows_a)
    assert np.array_equal(num.sum(axis=1), rows_b)
    for _ in range(4):
        v = rng.integers(-2, 3, size=pa).astype(np.int64)
        lhs = num @ v
        rhs = n * (b64.T @ (a64 @ v)) - sb * int(sa @ v)
        assert np.array_equal(lhs, rhs)
    # Gamma follows from the exact numerator by one FP64 division everywhere
    assert np.array_equal(got["gamma"], num.reshape(-1).astype(np.float64) / float(n * n))
    assert np.array_equal(got["gamma_f32"], got["gamma"].astype(np.float32))
    again = run_correlate(cpi, a, b, n, pa, pb, cpi.FRAMES_U8, cpi.GAMMA_VIEW_MAJOR)
    assert_bit_exact(again, got, "rerun ")
    del torch


def test_measured_peaks_plausible(cpi):
    """The device microbenchmarks report positive rates below the vendor peaks
    (with a little margin for clock variation)."""
    log("case measured peaks")
    mp = cpi.measure_peaks(copy_bytes=256 << 20)
    assert 0.5e15 < mp["int8_ops_per_s"] < 5.2e15
    assert 1.0e15 < mp["fp4_ops_per_s"] < 10.5e15
    assert 0.5e12 < mp["copy_bytes_per_s"] < 8.5e12


@pytest.mark.parametrize("fmt_name", ["bit1", "u8"])
def test_memory_adaptive_blocks(cpi, fmt_name):
    """A workspace below the single-shot plan makes cpi_correlate fold the
    frames in blocks (the largest multiple of 512 frames whose running-sum state
    fits); Gamma, the numerator and the sums are bit-identical to the
    single-shot call.  Also forced through CPI_WORKSPACE_LIMIT."""
    import os
    import torch
    rng = np.random.default_rng(77)
    n, pa, pb = 40000, 1024, 256
    if fmt_name == "bit1":
        fmt = cpi.FRAMES_BIT1
        fa = rng.integers(0, 256, (n, pa // 8), dtype=np.uint8)
        fb = rng.integers(0, 256, (n, pb // 8), dtype=np.uint8)
        limit = 3_000_000
    else:
        fmt = cpi.FRAMES_U8
        fa = rng.poisson(3.0, (n, pa)).clip(0, 255).astype(np.uint8)
        fb = rng.poisson(3.0, (n, pb)).clip(0, 255).astype(np.uint8)
        fa[7, 5] = 255
        limit = 8_000_000
    full = cpi.correlate_workspace_size(n, pa, pb, fmt)
    assert full > limit
    log(f"blocks {fmt_name}: single-shot workspace {full} bytes, limit {limit}")
    da, db = to_dev(fa), to_dev(fb)

    def run(ws_bytes):
        outs = dict(gamma=torch.empty(pa * pb, dtype=torch.float64, device=dev()),
                    gamma_f32=torch.empty(pa * pb, dtype=torch.float32, device=dev()),
                    numer=torch.empty(pa * pb, dtype=torch.int64, device=dev()),
                    sum_a=torch.empty(pa, dtype=torch.int64, device=dev()),
                    sum_b=torch.empty(pb, dtype=torch.int64, device=dev()))
        ws = cpi.alloc_workspace(ws_bytes, dev())
        cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR, workspace=ws, **outs)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in outs.items()}

    ref = run(full)
    got = run(limit)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
    os.environ["CPI_WORKSPACE_LIMIT"] = str(limit)
    try:
        need = cpi.correlate_workspace_size(n, pa, pb, fmt)
        assert need <= limit
        got2 = run(full)
    finally:
        del os.environ["CPI_WORKSPACE_LIMIT"]
    for k in ref:
        assert np.array_equal(ref[k], got2[k]), k
    # the numerator itself against the oracle's definition on a few entries
    q = rng.integers(0, pb, 6)
    p = rng.integers(0, pa, 6)
    of = oracle.FRAMES_BIT1 if fmt_name == "bit1" else oracle.FRAMES_U8
    A = oracle.unpack_frames(fa, n, pa, of)
    B = oracle.unpack_frames(fb, n, pb, of)
    for qq, pp in zip(q, p):
        a = A[:, pp].astype(np.int64)
        b = B[:, qq].astype(np.int64)
        num = n * int(a @ b) - int(a.sum()) * int(b.sum())
        assert ref["numer"][qq * pa + pp] == num
