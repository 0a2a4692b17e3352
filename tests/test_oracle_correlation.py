"""Pins of the correlation oracle (CPU only).

Each test ties the oracle to something other than itself: hand-worked examples
of Eq. (1), the definition evaluated in exact rational arithmetic, closed forms
for N = 1 and N = 2, the symmetry/diagonal/PSD structure when both detectors
see the same frames, integer row-sum identities, offset and permutation
invariances, Freivalds' check and a statistical bound for independent
detectors.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import pack_bits_lsb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _frames(hexes):
    return np.frombuffer(bytes.fromhex("".join(hexes)), dtype=np.uint8)


def _eq1_fraction(a, b):
    """Eq. (1) literally: mean of products minus product of means, exact."""
    n, pa = a.shape
    pb = b.shape[1]
    out = [[None] * pb for _ in range(pa)]
    for p in range(pa):
        for q in range(pb):
            mab = Fraction(sum(int(a[i, p]) * int(b[i, q]) for i in range(n)), n)
            ma = Fraction(sum(int(a[i, p]) for i in range(n)), n)
            mb = Fraction(sum(int(b[i, q]) for i in range(n)), n)
            out[p][q] = mab - ma * mb
    return out


@pytest.mark.parametrize("name", ["gamma_u8_3frames.json", "gamma_bit1_4frames.json",
                                  "gamma_u8_large_values.json"])
def test_hand_worked_examples(name):
    fx = _load(name)
    fmt = oracle.FRAMES_U8 if fx["fmt"] == "u8" else oracle.FRAMES_BIT1
    r = oracle.correlation(_frames(fx["frames_a_hex"]), _frames(fx["frames_b_hex"]),
                           fx["n"], fx["pa"], fx["pb"], fmt)
    assert r["sum_a"].tolist() == fx["sum_a"]
    assert r["sum_b"].tolist() == fx["sum_b"]
    assert r["numer"].tolist() == fx["numer"]
    want = np.array([[float(Fraction(v)) for v in row] for row in fx["gamma"]])
    assert np.array_equal(r["gamma"], want)


def test_unpack_bit_order():
    # byte 0b00000101 -> pixels 0 and 2; byte 0b00000010 -> pixel 9; 10 px/frame
    frames = np.array([0x05, 0x02], dtype=np.uint8)
    got = oracle.unpack_frames(frames, 1, 10, oracle.FRAMES_BIT1)
    assert got.tolist() == [[1, 0, 1, 0, 0, 0, 0, 0, 0, 1]]


@pytest.mark.parametrize("npix", [1, 7, 8, 9, 31, 64, 100])
def test_pack_unpack_roundtrip(npix):
    rng = np.random.default_rng(npix)
    x = (rng.random((5, npix)) < 0.4).astype(np.uint8)
    packed = pack_bits_lsb(x)
    assert packed.shape == (5, (npix + 7) // 8)
    assert np.array_equal(oracle.unpack_frames(packed, 5, npix, oracle.FRAMES_BIT1), x)


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_fraction_u8(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 9))
    pa = int(rng.integers(1, 17))
    pb = int(rng.integers(1, 17))
    a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
    b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
    r = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    ref = _eq1_fraction(a, b)
    for p in range(pa):
        for q in range(pb):
            assert r["numer"][p, q] == ref[p][q] * n * n
            assert r["gamma"][p, q] == float(ref[p][q])


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_fraction_bits(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 9))
    pa = int(rng.integers(1, 17))
    pb = int(rng.integers(1, 17))
    a = (rng.random((n, pa)) < 0.5).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.5).astype(np.uint8)
    r = oracle.correlation(pack_bits_lsb(a), pack_bits_lsb(b), n, pa, pb, oracle.FRAMES_BIT1)
    ref = _eq1_fraction(a, b)
    for p in range(pa):
        for q in range(pb):
            assert r["numer"][p, q] == ref[p][q] * n * n
            assert r["gamma"][p, q] == float(ref[p][q])


def test_single_frame_is_zero():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 256, size=(1, 40), dtype=np.uint8)
    b = rng.integers(0, 256, size=(1, 9), dtype=np.uint8)
    r = oracle.correlation(a, b, 1, 40, 9, oracle.FRAMES_U8)
    assert not r["numer"].any()
    assert not r["gamma"].any()


def test_two_frames_closed_form():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 256, size=(2, 33), dtype=np.uint8)
    b = rng.integers(0, 256, size=(2, 17), dtype=np.uint8)
    r = oracle.correlation(a, b, 2, 33, 17, oracle.FRAMES_U8)
    da = a[0].astype(np.int64) - a[1]
    db = b[0].astype(np.int64) - b[1]
    assert np.array_equal(r["numer"], np.outer(da, db))
    assert np.array_equal(r["gamma"], np.outer(da, db) / 4.0)


@pytest.mark.parametrize("bits", [True, False])
def test_same_detector_symmetry_diagonal_psd(bits):
    rng = np.random.default_rng(5)
    n, p = 300, 48
    if bits:
        a = (rng.random((n, p)) < 0.3).astype(np.uint8)
    else:
        a = rng.integers(0, 256, size=(n, p), dtype=np.uint8)
    r = oracle.correlation(a, a, n, p, p, oracle.FRAMES_U8)
    num = r["numer"]
    assert np.array_equal(num, num.T)
    s = a.sum(axis=0, dtype=np.int64)
    sq = (a.astype(np.int64) ** 2).sum(axis=0)
    assert np.array_equal(np.diag(num), n * sq - s * s)
    if bits:
        assert np.array_equal(np.diag(num), s * (n - s))
    ev = np.linalg.eigvalsh(r["gamma"])
    assert ev.min() > -1e-9 * max(1.0, ev.max())


def test_row_and_column_sum_identities():
    rng = np.random.default_rng(6)
    n, pa, pb = 777, 130, 70
    a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
    b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
    r = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    a64 = a.astype(np.int64)
    b64 = b.astype(np.int64)
    tb = b64.sum(axis=1)            # |B_i|
    ta = a64.sum(axis=1)            # |A_i|
    sa = a64.sum(axis=0)
    sb = b64.sum(axis=0)
    rows = n * (a64 * tb[:, None]).sum(axis=0) - sa * sb.sum()
    cols = n * (b64 * ta[:, None]).sum(axis=0) - sb * sa.sum()
    assert np.array_equal(r["numer"].sum(axis=1), rows)
    assert np.array_equal(r["numer"].sum(axis=0), cols)
    assert r["numer"].sum() == n * int((ta * tb).sum()) - int(sa.sum()) * int(sb.sum())


def test_offset_invariance():
    rng = np.random.default_rng(7)
    n, pa, pb = 200, 25, 11
    a = rng.integers(0, 100, size=(n, pa), dtype=np.uint8)
    b = rng.integers(0, 100, size=(n, pb), dtype=np.uint8)
    r0 = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    r1 = oracle.correlation(a + 128, b + 37, n, pa, pb, oracle.FRAMES_U8)
    assert np.array_equal(r0["numer"], r1["numer"])
    assert np.array_equal(r0["gamma"], r1["gamma"])


def test_permutation_and_chunk_invariance():
    rng = np.random.default_rng(8)
    n, pa, pb = 1000, 40, 20
    a = (rng.random((n, pa)) < 0.2).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.2).astype(np.uint8)
    whole = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    perm = rng.permutation(n)
    shuf = oracle.correlation(a[perm], b[perm], n, pa, pb, oracle.FRAMES_U8)
    assert np.array_equal(whole["numer"], shuf["numer"])
    # streaming: fold chunk sums, then form the numerator once
    s_ab = np.zeros((pa, pb), dtype=np.int64)
    s_a = np.zeros(pa, dtype=np.int64)
    s_b = np.zeros(pb, dtype=np.int64)
    for lo, hi in [(0, 1), (1, 300), (300, 301), (301, 1000)]:
        c = oracle.correlation(a[lo:hi], b[lo:hi], hi - lo, pa, pb, oracle.FRAMES_U8)
        k = hi - lo
        # numer_c = k S_ab,c - S_a,c S_b,c  =>  S_ab,c = (numer_c + S_a,c S_b,c) / k
        s_ab += (c["numer"] + np.outer(c["sum_a"], c["sum_b"])) // k
        s_a += c["sum_a"]
        s_b += c["sum_b"]
    assert np.array_equal(n * s_ab - np.outer(s_a, s_b), whole["numer"])


def test_freivalds_moderate_size():
    rng = np.random.default_rng(9)
    n, pa, pb = 3000, 600, 150
    a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
    b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
    r = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    a64 = a.astype(np.int64)
    b64 = b.astype(np.int64)
    for _ in range(8):
        v = rng.integers(-3, 4, size=pb).astype(np.int64)
        lhs = r["numer"] @ v
        rhs = n * (a64.T @ (b64 @ v)) - a64.sum(axis=0) * int(b64.sum(axis=0) @ v)
        assert np.array_equal(lhs, rhs)


def test_subset_rows_match_full():
    rng = np.random.default_rng(10)
    n, pa, pb = 500, 64, 32
    a = (rng.random((n, pa)) < 0.1).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.1).astype(np.uint8)
    full = oracle.correlation(pack_bits_lsb(a), pack_bits_lsb(b), n, pa, pb, oracle.FRAMES_BIT1)
    rows = np.array([0, 5, 63])
    cols = np.array([31, 2])
    sub = oracle.correlation(pack_bits_lsb(a), pack_bits_lsb(b), n, pa, pb,
                             oracle.FRAMES_BIT1, rows_a=rows, cols_b=cols)
    assert np.array_equal(sub["numer"], full["numer"][np.ix_(rows, cols)])


def test_independent_detectors_statistics():
    """Independent detectors: Gamma / sqrt(var_a var_b / N) is ~N(0,1)."""
    rng = np.random.default_rng(11)
    n, pa, pb = 20000, 128, 128
    a = (rng.random((n, pa)) < 0.1).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.1).astype(np.uint8)
    r = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    ma = r["sum_a"] / n
    mb = r["sum_b"] / n
    va = ma - ma * ma
    vb = mb - mb * mb
    z = r["gamma"] / np.sqrt(np.outer(va, vb) / n)
    assert abs(z.mean()) < 5.0 / np.sqrt(pa * pb)
    assert np.abs(z).max() < np.sqrt(2 * np.log(pa * pb)) + 1.5
    assert 0.9 < z.std() < 1.1


def test_overflow_bound():
    assert oracle.overflow_ok(20000, 1, 1)
    assert oracle.overflow_ok(11_000_000, 255, 255)
    assert not oracle.overflow_ok(12_000_000, 255, 255)
    assert oracle.overflow_ok(94_000_000, 1, 1)
    assert not oracle.overflow_ok(95_000_000, 1, 1)


def test_layouts():
    x = np.arange(6).reshape(2, 3)
    assert oracle.to_layout(x, oracle.GAMMA_PIXEL_MAJOR).tolist() == x.tolist()
    assert oracle.to_layout(x, oracle.GAMMA_VIEW_MAJOR).tolist() == x.T.tolist()
