"""GPU parity of the streaming path: chunks folded into device-resident sums
must give the single-shot oracle's Gamma bit for bit, after any chunking,
through a checkpoint and across encodings."""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, alphas_for, generate_frames, pack_bits_lsb
from tests.gpu_util import assert_bit_exact, dev, log, oracle_in_layout, plane_rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpi():
    import paper_2407_20692_amd as m
    return m


def _gamma(cpi, s, layout=oracle.GAMMA_VIEW_MAJOR):
    import torch

    d = dev()
    n = s.pa * s.pb
    out = {
        "gamma": torch.empty(n, dtype=torch.float64, device=d),
        "gamma_f32": torch.empty(n, dtype=torch.float32, device=d),
        "numer": torch.empty(n, dtype=torch.int64, device=d),
        "sum_a": torch.empty(s.pa, dtype=torch.int64, device=d),
        "sum_b": torch.empty(s.pb, dtype=torch.int64, device=d),
    }
    s.gamma(layout, **out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _chunks(n, sizes):
    lo = 0
    for k in sizes:
        if lo >= n:
            break
        yield lo, min(n, lo + k)
        lo += k


@pytest.mark.parametrize("enc", ["auto", "int8"])
@pytest.mark.parametrize("fmt_name", ["bit1", "u8_binary", "u8_counts"])
def test_chunked_equals_single_shot(cpi, fmt_name, enc):
    """Chunks of every format folded into the running sums equal the oracle's
    single shot, under either matrix-core encoding of binary chunks."""
    before = cpi.get_mma_encoding()
    cpi.set_mma_encoding(cpi.MMA_INT8 if enc == "int8" else cpi.MMA_AUTO)
    try:
        _chunked_equals_single_shot(cpi, fmt_name, enc)
    finally:
        cpi.set_mma_encoding(before)


def _chunked_equals_single_shot(cpi, fmt_name, enc):
    rng = np.random.default_rng(21)
    n, pa, pb = 5000, 300, 70
    if fmt_name == "u8_counts":
        a = rng.integers(0, 256, size=(n, pa), dtype=np.uint8)
        b = rng.integers(0, 256, size=(n, pb), dtype=np.uint8)
        a[:2000] //= 128     # early chunks stay binary, later ones do not
        b[:2000] //= 128
    else:
        a = (rng.random((n, pa)) < 0.2).astype(np.uint8)
        b = (rng.random((n, pb)) < 0.2).astype(np.uint8)
    fmt = cpi.FRAMES_BIT1 if fmt_name == "bit1" else cpi.FRAMES_U8
    s = cpi.Stream(pa, pb, fmt, max_chunk=1200)
    for lo, hi in _chunks(n, [1000, 1, 1200, 999, 64, 1136, 600]):
        ca = pack_bits_lsb(a[lo:hi]) if fmt_name == "bit1" else a[lo:hi]
        cb = pack_bits_lsb(b[lo:hi]) if fmt_name == "bit1" else b[lo:hi]
        log(f"case stream {fmt_name} encoding={enc} chunk [{lo},{hi})")
        s.push(to_dev(ca), to_dev(cb), hi - lo)
    assert s.frames == n
    ref = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    for layout in (oracle.GAMMA_VIEW_MAJOR, oracle.GAMMA_PIXEL_MAJOR):
        assert_bit_exact(_gamma(cpi, s, layout), oracle_in_layout(ref, layout))
    s.close()


def test_checkpoint_resume(cpi):
    rng = np.random.default_rng(22)
    n, pa, pb = 4000, 256, 64
    a = (rng.random((n, pa)) < 0.1).astype(np.uint8)
    b = (rng.random((n, pb)) < 0.1).astype(np.uint8)
    pa_bits, pb_bits = pack_bits_lsb(a), pack_bits_lsb(b)
    s1 = cpi.Stream(pa, pb, cpi.FRAMES_BIT1, max_chunk=1000)
    for lo in range(0, 2000, 1000):
        s1.push(to_dev(pa_bits[lo:lo + 1000]), to_dev(pb_bits[lo:lo + 1000]), 1000)
    log("case checkpoint save/load")
    state = s1.save()
    s1.close()
    s2 = cpi.Stream(pa, pb, cpi.FRAMES_BIT1, max_chunk=1000)
    s2.load(state)
    assert s2.frames == 2000
    for lo in range(2000, n, 1000):
        s2.push_host(pa_bits[lo:lo + 1000], pb_bits[lo:lo + 1000], 1000)
    ref = oracle.correlation(a, b, n, pa, pb, oracle.FRAMES_U8)
    assert_bit_exact(_gamma(cpi, s2), oracle_in_layout(ref, oracle.GAMMA_VIEW_MAJOR))
    s2.close()


def test_stream_gamma_f32_and_refocus_after_each_chunk(cpi):
    import torch

    w = WORKLOADS["da32_db16_n1000_u8counts"]
    rng = np.random.default_rng(23)
    n = 3000
    a = (rng.random((n, w.pa)) < 0.15).astype(np.uint8)
    b = (rng.random((n, w.pb)) < 0.15).astype(np.uint8)
    s = cpi.Stream(w.pa, w.pb, cpi.FRAMES_BIT1, max_chunk=1000)
    g = cpi.geometry_default(w.wa, w.ha, w.wb, w.hb)
    og = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    al = alphas_for(w)
    out = torch.empty(len(al) * w.pa, dtype=torch.float32, device=dev())
    for lo in range(0, n, 1000):
        s.push(to_dev(pack_bits_lsb(a[lo:lo + 1000])), to_dev(pack_bits_lsb(b[lo:lo + 1000])), 1000)
        s.refocus(g, al, out)
        torch.cuda.synchronize()
        m = lo + 1000
        log(f"case stream refocus after {m} frames")
        ref = oracle.correlation(a[:m], b[:m], m, w.pa, w.pb, oracle.FRAMES_U8)
        g32 = torch.empty(w.pa * w.pb, dtype=torch.float32, device=dev())
        s.gamma(cpi.GAMMA_VIEW_MAJOR, gamma_f32=g32)
        torch.cuda.synchronize()
        want32 = oracle.to_layout(ref["gamma_f32"], oracle.GAMMA_VIEW_MAJOR).reshape(-1)
        assert np.array_equal(g32.cpu().numpy(), want32)
        want = oracle.refocus(oracle.to_layout(ref["gamma"], oracle.GAMMA_VIEW_MAJOR), og, al)
        got = out.cpu().numpy().reshape(want.shape)
        assert plane_rel_err(got, want).max() <= 1e-5
    s.close()


def test_stream_errors(cpi):
    s = cpi.Stream(64, 16, cpi.FRAMES_BIT1, max_chunk=100)
    import torch

    with pytest.raises(cpi.CpiError) as e:
        s.gamma(cpi.GAMMA_VIEW_MAJOR, gamma=torch.empty(64 * 16, dtype=torch.float64, device=dev()))
    assert e.value.status == 6   # not ready
    x = torch.zeros(200 * 8, dtype=torch.uint8, device=dev())
    with pytest.raises(cpi.CpiError) as e:
        s.push(x, x, 101)
    assert e.value.status == 1
    s.close()


def test_streaming_workload_final_gamma(cpi):
    """Da 128x128, Db 64x64, 1-bit frames in chunks of 1000 (first 40 chunks
    of the streamed workload): final Gamma checked on 64 sampled views against
    the single-shot oracle, plus exact row/column sums of the numerator."""
    import torch

    w = WORKLOADS["da128_db64_stream200x1000_bit1"]
    n = 40000
    a, b = generate_frames(w, count=n)
    s = cpi.Stream(w.pa, w.pb, cpi.FRAMES_BIT1, max_chunk=w.chunk)
    pa_bits, pb_bits = pack_bits_lsb(a), pack_bits_lsb(b)
    for lo in range(0, n, w.chunk):
        s.push(to_dev(pa_bits[lo:lo + w.chunk]), to_dev(pb_bits[lo:lo + w.chunk]), w.chunk)
    log(f"case {w.name} first {n} frames")
    got = _gamma(cpi, s)
    num = got["numer"].reshape(w.pb, w.pa)
    views = np.sort(np.random.default_rng(5).choice(w.pb, 64, replace=False))
    ref = oracle.correlation(a, b, n, w.pa, w.pb, oracle.FRAMES_U8, cols_b=views)
    assert np.array_equal(num[views], ref["numer"].T)
    assert np.array_equal(got["gamma"].reshape(w.pb, w.pa)[views], ref["gamma"].T)
    a64, b64 = a.astype(np.int64), b.astype(np.int64)
    sa, sb = a64.sum(0), b64.sum(0)
    rows_a = n * (a64 * b64.sum(1)[:, None]).sum(0) - sa * sb.sum()
    assert np.array_equal(num.sum(axis=0), rows_a)
    s.close()
    del torch


def _columns(packed, pix):
    """0/1 values of the listed pixels in every frame, from packed bytes (host)."""
    pix = np.asarray(pix)
    return ((packed[:, pix // 8] >> (pix % 8)) & 1).astype(np.uint8)


def test_streaming_workload_200_distinct_chunks(cpi):
    """The whole streamed workload: Da 128x128, Db 64x64, 200 distinct seeded
    chunks of 1000 1-bit frames (made on the device), folded one by one up to
    N = 200000.  The final state equals single-shot correlation of the same
    frames bit for bit over every entry; sampled entries equal the oracle's;
    every row and column sum of the numerator and a Freivalds product equal
    their values computed from the frames (exact integers in FP64)."""
    import torch
    from synth.gpu_speckle import generate_binary_frames_gpu

    w = WORKLOADS["da128_db64_stream200x1000_bit1"]
    n, pa, pb, k = w.n_frames, w.pa, w.pb, w.chunk
    d = dev()
    log(f"case {w.name}: generating {n} frames on the device")
    fa, fb = generate_binary_frames_gpu(w, count=n, device=d)
    s = cpi.Stream(pa, pb, cpi.FRAMES_BIT1, max_chunk=k)
    for c in range(n // k):
        s.push(fa[c * k:(c + 1) * k].reshape(-1), fb[c * k:(c + 1) * k].reshape(-1), k)
        if c % 50 == 49:
            torch.cuda.synchronize()
            log(f"case {w.name}: {c + 1} chunks folded")
    assert s.frames == n
    st = {
        "gamma": torch.empty(pa * pb, dtype=torch.float64, device=d),
        "gamma_f32": torch.empty(pa * pb, dtype=torch.float32, device=d),
        "numer": torch.empty(pa * pb, dtype=torch.int64, device=d),
        "sum_a": torch.empty(pa, dtype=torch.int64, device=d),
        "sum_b": torch.empty(pb, dtype=torch.int64, device=d),
    }
    s.gamma(cpi.GAMMA_VIEW_MAJOR, **st)
    one = {key: torch.empty_like(v) for key, v in st.items()}
    log(f"case {w.name}: single shot")
    cpi.correlate(fa.reshape(-1), fb.reshape(-1), n, pa, pb, cpi.FRAMES_BIT1,
                  cpi.GAMMA_VIEW_MAJOR, **one)
    torch.cuda.synchronize()
    s.close()
    for key in st:
        assert torch.equal(st[key], one[key]), key
    # sampled entries against the oracle (from the sampled pixels' frame columns)
    rng = np.random.default_rng(24)
    rows = np.sort(rng.choice(pa, 1024, replace=False))
    views = np.sort(rng.choice(pb, 64, replace=False))
    ha, hb = fa.cpu().numpy(), fb.cpu().numpy()
    ref = oracle.correlation(_columns(ha, rows), _columns(hb, views), n, rows.size, views.size,
                             oracle.FRAMES_U8)
    num = st["numer"].view(pb, pa)
    assert np.array_equal(num[views][:, rows].cpu().numpy(), ref["numer"].T)
    assert np.array_equal(st["gamma"].view(pb, pa)[views][:, rows].cpu().numpy(), ref["gamma"].T)
    assert np.array_equal(st["sum_a"].cpu().numpy()[rows], ref["sum_a"])
    assert np.array_equal(st["sum_b"].cpu().numpy()[views], ref["sum_b"])
    # identities over every entry, from the frames (integers below 2^53 in FP64)
    log(f"case {w.name}: row/column sums and Freivalds")
    bits = torch.arange(8, device=d, dtype=torch.uint8)

    def unpacked(packed, npix, step=20000):
        for lo in range(0, packed.shape[0], step):
            c = packed[lo:lo + step]
            yield lo, ((c.unsqueeze(2) >> bits) & 1).reshape(c.shape[0], -1)[:, :npix]

    ta = torch.zeros(n, dtype=torch.float64, device=d)
    tb = torch.zeros(n, dtype=torch.float64, device=d)
    for lo, u in unpacked(fa, pa):
        ta[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    for lo, u in unpacked(fb, pb):
        tb[lo:lo + u.shape[0]] = u.sum(dim=1, dtype=torch.float64)
    v = torch.from_numpy(rng.integers(-2, 3, size=pa).astype(np.float64)).to(d)
    a_tb = torch.zeros(pa, dtype=torch.float64, device=d)
    a_v = torch.zeros(n, dtype=torch.float64, device=d)
    sa_f = torch.zeros(pa, dtype=torch.float64, device=d)
    for lo, u in unpacked(fa, pa):
        uf = u.to(torch.float64)
        a_tb += uf.t() @ tb[lo:lo + u.shape[0]]
        a_v[lo:lo + u.shape[0]] = uf @ v
        sa_f += uf.sum(dim=0)
    b_ta = torch.zeros(pb, dtype=torch.float64, device=d)
    bt_av = torch.zeros(pb, dtype=torch.float64, device=d)
    sb_f = torch.zeros(pb, dtype=torch.float64, device=d)
    for lo, u in unpacked(fb, pb):
        uf = u.to(torch.float64)
        b_ta += uf.t() @ ta[lo:lo + u.shape[0]]
        bt_av += uf.t() @ a_v[lo:lo + u.shape[0]]
        sb_f += uf.sum(dim=0)
    assert torch.equal(sa_f, st["sum_a"].to(torch.float64))
    assert torch.equal(sb_f, st["sum_b"].to(torch.float64))
    numf = num.to(torch.float64)
    assert torch.equal(numf.sum(dim=0), n * a_tb - sa_f * sb_f.sum())
    assert torch.equal(numf.sum(dim=1), n * b_ta - sb_f * sa_f.sum())
    assert torch.equal(numf @ v, n * bt_av - sb_f * (sa_f @ v))


@pytest.mark.parametrize("buffers", [2, 1])
def test_overlapped_refocus_matches_serial(cpi, buffers):
    """The streamed workload (Da 128x128, Db 64x64, 200 distinct chunks of 1000
    1-bit frames) with the refocus of chunk k enqueued on a second stream while
    chunk k + 1 is folded on the handle's stream (two FP32 Gamma buffers; one
    buffer serialises the two and must give the same results).  Every chunk's
    refocused stack equals the serial stream's bit for bit, and the final state
    equals single-shot correlation of all 200000 frames over every entry."""
    import torch
    from synth.gpu_speckle import generate_binary_frames_gpu

    w = WORKLOADS["da128_db64_stream200x1000_bit1"]
    n, pa, pb, k = w.n_frames, w.pa, w.pb, w.chunk
    nch = n // k if buffers == 2 else 20
    d = dev()
    log(f"case {w.name}: {nch} chunks, {buffers} Gamma buffers")
    fa, fb = generate_binary_frames_gpu(w, count=nch * k, device=d)
    geo = cpi.geometry_default(w.wa, w.ha, w.wb, w.hb)
    al = alphas_for(w)
    na = len(al)
    need = cpi.refocus_workspace_size(geo, na)
    ser = cpi.Stream(pa, pb, cpi.FRAMES_BIT1, max_chunk=k)
    out_s = torch.empty((nch, na * pa), dtype=torch.float32, device=d)
    ws_s = cpi.alloc_workspace(need, d)
    for c in range(nch):
        ser.push(fa[c * k:(c + 1) * k].reshape(-1), fb[c * k:(c + 1) * k].reshape(-1), k)
        ser.refocus(geo, al, out_s[c], workspace=ws_s)
    torch.cuda.synchronize()
    su, sr = torch.cuda.Stream(), torch.cuda.Stream()
    ovl = cpi.Stream(pa, pb, cpi.FRAMES_BIT1, max_chunk=k, stream=su, gamma_buffers=buffers)
    out_o = torch.full((nch, na * pa), float("nan"), dtype=torch.float32, device=d)
    ws_o = cpi.alloc_workspace(need, d)
    torch.cuda.synchronize()
    for c in range(nch):
        ovl.push(fa[c * k:(c + 1) * k].reshape(-1), fb[c * k:(c + 1) * k].reshape(-1), k)
        ovl.refocus_async(geo, al, out_o[c], ws_o, sr)
    torch.cuda.synchronize()
    assert ovl.frames == nch * k
    bad = [c for c in range(nch) if not torch.equal(out_o[c], out_s[c])]
    assert not bad, f"chunks whose stacks differ: {bad[:10]}"
    keys = ("gamma", "gamma_f32", "numer", "sum_a", "sum_b")
    sizes = {"gamma": (pa * pb, torch.float64), "gamma_f32": (pa * pb, torch.float32),
             "numer": (pa * pb, torch.int64), "sum_a": (pa, torch.int64), "sum_b": (pb, torch.int64)}
    got = {key: torch.empty(sizes[key][0], dtype=sizes[key][1], device=d) for key in keys}
    ovl.gamma(cpi.GAMMA_VIEW_MAJOR, **got)
    torch.cuda.synchronize()
    one = {key: torch.empty_like(v) for key, v in got.items()}
    cpi.correlate(fa.reshape(-1), fb.reshape(-1), nch * k, pa, pb, cpi.FRAMES_BIT1,
                  cpi.GAMMA_VIEW_MAJOR, **one)
    torch.cuda.synchronize()
    for key in keys:
        assert torch.equal(got[key], one[key]), key
    ser.close()
    ovl.close()


def test_overlapped_stream_errors(cpi):
    import torch

    with pytest.raises(cpi.CpiError) as e:
        cpi.Stream(64, 16, cpi.FRAMES_BIT1, max_chunk=100, gamma_buffers=3)
    assert e.value.status == 1
    s = cpi.Stream(64, 16, cpi.FRAMES_BIT1, max_chunk=100, gamma_buffers=2)
    geo = cpi.geometry_default(8, 8, 4, 4)
    out = torch.empty(64, dtype=torch.float32, device=dev())
    ws = cpi.alloc_workspace(cpi.refocus_workspace_size(geo, 1), dev())
    with pytest.raises(cpi.CpiError) as e:
        s.refocus_async(geo, [1.0], out, ws, torch.cuda.Stream())
    assert e.value.status == 6   # not ready
    s.close()


def test_host_pushes_from_pinned_memory(cpi):
    """Host chunks from pinned memory (copies on the handle's copy stream,
    alternating staging buffers, no host waits between pushes), u8 and 1-bit,
    with ragged chunk sizes: the final state equals pushes of the same chunks
    from device memory bit for bit, and the FP32 Gamma after each push equals
    the device-push stream's."""
    import torch

    rng = np.random.default_rng(31)
    for fmt_name in ("bit1", "u8"):
        n, pa, pb = 6000, 256, 64
        a = (rng.random((n, pa)) < 0.25).astype(np.uint8)
        b = (rng.random((n, pb)) < 0.25).astype(np.uint8)
        fmt = cpi.FRAMES_BIT1 if fmt_name == "bit1" else cpi.FRAMES_U8
        fa = pack_bits_lsb(a) if fmt_name == "bit1" else a
        fb = pack_bits_lsb(b) if fmt_name == "bit1" else b
        ha = torch.from_numpy(np.ascontiguousarray(fa)).pin_memory()
        hb = torch.from_numpy(np.ascontiguousarray(fb)).pin_memory()
        sh = cpi.Stream(pa, pb, fmt, max_chunk=1100)
        sd = cpi.Stream(pa, pb, fmt, max_chunk=1100)
        g_h, g_d = [], []
        for lo, hi in _chunks(n, [1000, 7, 1100, 513, 999, 1100, 64, 1100, 117]):
            log(f"case host push {fmt_name} frames {lo}..{hi}")
            sh.push_host(ha[lo:hi].reshape(-1), hb[lo:hi].reshape(-1), hi - lo)
            sd.push(to_dev(fa[lo:hi]), to_dev(fb[lo:hi]), hi - lo)
            x = torch.empty(pa * pb, dtype=torch.float32, device=dev())
            y = torch.empty_like(x)
            sh.gamma(cpi.GAMMA_VIEW_MAJOR, gamma_f32=x)
            sd.gamma(cpi.GAMMA_VIEW_MAJOR, gamma_f32=y)
            g_h.append(x)
            g_d.append(y)
        torch.cuda.synchronize()
        for x, y in zip(g_h, g_d):
            assert torch.equal(x, y)
        assert_bit_exact(_gamma(cpi, sh), _gamma(cpi, sd))
        sh.close()
        sd.close()
