#!/usr/bin/env python3
"""Benchmark of the correlation plenoptic imaging hot path on one MI355X.

Default workload (the headline line): Da 256x256, Db 128x128, N = 100000
distinct 1-bit frames packed 8 per byte (seeded speckle through a 3-slit mask,
SPAD-like occupancy ~0.1, generated on the device), 128 refocus planes alpha
in [0.5, 1.5].  One step is one pass of the hot path with the inputs resident
in HBM: ingest + matrix-core contraction with the exact int64/FP64 epilogue
(Gamma in FP64 and FP32) + batched refocus of all planes with the autotuned
configuration (tuned once before timing).  Binary frames are contracted as FP4
(E2M1) 0/1 operands with FP32 sums, exact below 2^24 frames per pass; the int8
encoding of the same step is timed beside it.

Printed as ONE JSON line:
  value          Gamma pixel-pair*frames per second over the whole step
                 (N * Pa * Pb per step / step time), FP4 encoding
  correlate, refocus  per-kernel-group times of the step (library events)
  int8_step      the same step with the int8 encoding of the contraction
  fp32_plain     the plain FP32 path on the same inputs (correlator and
                 one-plane-per-launch refocus, the latter timed on 8 planes
                 and scaled to the stack) and the ratios to it
  roofline       the contraction kernel (dominant in the correlator) against
                 the FP4 peak, its duration measured with the library's HIP
                 events on its launch stream
  roofline_int8  the same contraction in the int8 encoding against the int8 peak
  roofline_refocus  the batched refocus kernel against the FP32 vector-ALU
                 peak (two FLOPs per bilinear tap), with its measured HBM and
                 LDS traffic where counter summaries exist for the current source
  cpu_baseline   the CPU oracle on a bounded sample of the workload,
                 extrapolated linearly (the sample is stated)
  paper_like     the same figures for Da 128x128, Db 64x64, N = 20000 binary
                 bytes, 32 planes
  streaming      chunk-to-stack latency p50/p99 and frames/s for 200 distinct
                 1000-frame 1-bit chunks (Da 128x128, Db 64x64), each pushed
                 from pinned host memory and followed by a 32-plane refocus
  refocus_plane_counts  the paper's stack sizes (100, 261, 1000 planes)
  refocus_resampled  refocusing with the lens plane sampled at half-pixel steps
                 (general 4-D multilinear interpolation): view resampling + refocus
  file_ingest    raw side-by-side frame files (the paper's 256 x 512 layout,
                 11 files of 512 frames) streamed into the running sums
  denoiser       the learned denoiser's training step (16 planes of 128 x 128)
                 and inference (32 planes): time and algorithmic BF16 FLOP rate
  measured_peaks the device's sustained matrix-core and copy rates (microbenchmarks)
"""
import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "da128_db64_n20000_u8bin"
LARGE_WORKLOAD = "da256_db128_n100000_bit1"
PAPER_WORKLOAD = "da256_db256_files11_bit1"
STREAM_WORKLOAD = "da128_db64_stream200x1000_bit1"
DENOISE_WORKLOAD = "da128_db64_denoise500to50000_bit1"
BF16_PEAK = 2.5e15          # dense bfloat16 matrix-core FLOP/s, MI355X
INT8_PEAK = 5.0e15          # dense int8 matrix-core ops/s, MI355X
FP4_PEAK = 10.1e15          # dense FP4 (and FP6) matrix-core ops/s, MI355X
FP32_VECTOR_PEAK = 157.3e12  # FP32 vector FLOP/s, MI355X (packed FP32 FMA)
FP32_UNPACKED_PEAK = 78.6e12  # FP32 vector FLOP/s with one FMA per lane per cycle
# LDS read bandwidth for 8- and 16-byte reads: 256 bytes per clock per CU,
# 256 CUs, 2.4 GHz (a microbenchmark of conflict-free ds_read_b64 / b128 on
# this part sustains 220-236 bytes per clock per CU; the paired and 4-byte
# forms run at half that)
LDS_PEAK = 256 * 256 * 2.4e9
# workload keys of the committed counter summaries (contraction, refocus)
PAPER_LIKE_KEY = ("da128_db64_n20000", "da128_db64_32planes")
LARGE_KEY = ("da256_db128_n100000", "da256_db128_128planes")
GEMM_SOURCE = os.path.join(ROOT, "paper_2407_20692_amd", "csrc", "kernels_gemm.hip")
REF_SOURCE = os.path.join(ROOT, "paper_2407_20692_amd", "csrc", "kernels_refocus.hip")
ROWS_SOURCE = os.path.join(ROOT, "paper_2407_20692_amd", "csrc", "kernels_refocus_rows.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _summary_fields(summary, source):
    """key: value fields of a committed counter summary, if it was taken on the
    current kernel source; else None."""
    if summary is None:
        return None
    fields = {}
    try:
        with open(summary) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
    except OSError:
        return None
    if fields.get("kernel_source_sha256_16") != source_hash(source):
        return None
    return fields


def _summary_value(summary, source, key, tiles=None):
    fields = _summary_fields(summary, source)
    if fields is None:
        return None
    if tiles is not None:
        key = key + "_tiles " + " ".join(str(int(v)) for v in tiles)
    try:
        return float(fields[key].split()[0])
    except (KeyError, ValueError, IndexError):
        return None


def measured_traffic(summary, source, tiles=None):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from a
    committed counter summary taken on the current kernel source (and, for the
    refocus, with these tiles); else None."""
    return _summary_value(summary, source, "hbm_bytes_per_launch", tiles)


def measured_lds(summary, source, tiles=None):
    """LDS bytes read per launch from the same kind of summary; else None."""
    return _summary_value(summary, source, "lds_read_bytes_per_launch", tiles)


def refocus_algorithmic_bytes(geo, alphas):
    """Bytes a refocus launch must move at least: per plane, 4 bytes for every
    Gamma element with a nonzero bilinear weight for some output pixel (the
    plane's footprint, counted exactly; separable per view into columns x
    rows), plus 4 bytes per output pixel written."""
    import numpy as np

    def taps(alpha, n_out, n_b, size, mag, ca, cb):
        xr = np.arange(n_out, dtype=np.float64)
        xb = np.arange(n_b, dtype=np.float64)
        u = (alpha * (xr[None, :] - ca) + ca) + (1.0 - alpha) * mag * (xb[:, None] - cb)
        x0 = np.floor(u)
        f = u - x0
        counts = np.zeros(n_b, dtype=np.int64)
        for i in range(n_b):
            sel = np.concatenate([x0[i][(1.0 - f[i]) > 0], (x0[i] + 1)[f[i] > 0]])
            sel = sel[(sel >= 0) & (sel < size)]
            counts[i] = np.unique(sel).size
        return counts.sum()

    total = 0
    for al in alphas:
        nx = taps(al, geo.out_w, geo.wb, geo.wa, geo.mag_x, geo.ca_x, geo.cb_x)
        ny = taps(al, geo.out_h, geo.hb, geo.ha, geo.mag_y, geo.ca_y, geo.cb_y)
        total += 4 * nx * ny + 4 * geo.out_w * geo.out_h
    return int(total)


def file_ingest_bench(cpi, torch, np, dev, n_files=11, roi=128):
    """Raw-frame file streaming at the paper's layout: n_files files of 512
    frames of 256 x 512 1-bit pixels (random clicks at occupancy 0.1), the
    roi x roi region of both halves folded into the running sums, one file per
    piece; wall time from the first read to the device finishing."""
    import tempfile

    f = cpi.sidebyside(512, 256, 64, 64, roi, roi)
    rng = np.random.default_rng(7)
    block = np.packbits((rng.random((512, 256 * 512)) < 0.1).astype(np.uint8), axis=1,
                        bitorder="little")
    d = tempfile.mkdtemp(prefix="cpi_frames_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    paths = []
    try:
        for i in range(n_files):
            pth = os.path.join(d, f"frames_{i:05d}.bin")
            block.tofile(pth)
            paths.append(pth)
        st = cpi.Stream(f.roi_pixels, f.roi_pixels, cpi.FRAMES_BIT1, max_chunk=512, device=dev)
        ha = torch.empty(512 * f.frame_bytes, dtype=torch.uint8).pin_memory()
        hb = torch.empty(512 * f.frame_bytes, dtype=torch.uint8).pin_memory()
        raw = torch.empty(512 * f.frame_bytes, dtype=torch.uint8, device=dev)
        st.ingest_files(paths[:1], f, ha, hb, raw)       # warm-up
        torch.cuda.synchronize()
        st2 = cpi.Stream(f.roi_pixels, f.roi_pixels, cpi.FRAMES_BIT1, max_chunk=512, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = st2.ingest_files(paths, f, ha, hb, raw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st.close()
        st2.close()
    finally:
        for pth in paths:
            os.remove(pth)
        os.rmdir(d)
    return {"files": n_files, "frames": k, "frame": "256 x 512 px, 1 bit, A left / B right",
            "roi": [roi, roi], "seconds": t, "frames_per_s": k / t,
            "raw_MB_per_s": k * f.frame_bytes / t / 1e6}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_baseline(a, b, w, alphas):
    """The oracle, as it stands, on a bounded sample of the paper-like
    workload (about 12 s of host work): Gamma for every pixel pair over all
    frames, and 10 of the refocus planes (evenly spaced, first and last
    included)."""
    import numpy as np

    import oracle

    threads = _blas_threads()
    t0 = time.perf_counter()
    r = oracle.correlation(a, b, w.n_frames, w.pa, w.pb, oracle.FRAMES_U8)
    t1 = time.perf_counter()
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    gam = oracle.to_layout(r["gamma"], oracle.GAMMA_VIEW_MAJOR)
    del r
    planes = np.unique(np.linspace(0, len(alphas) - 1, 10).round().astype(int))
    t2 = time.perf_counter()
    oracle.refocus(gam, g, np.asarray(alphas)[planes])
    t3 = time.perf_counter()
    corr_rate = float(w.n_frames) * w.pa * w.pb / (t1 - t0)
    return {
        "value": corr_rate,
        "unit": "pixel-pair*frames/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"Gamma of all {w.pa} x {w.pb} pixel pairs over {w.n_frames} frames "
                   f"({t1 - t0:.2f} s); refocus of {planes.size} of {len(alphas)} planes "
                   f"({t3 - t2:.2f} s)"),
        "refocus_planes_per_s": planes.size / (t3 - t2),
        "seconds": (t1 - t0) + (t3 - t2),
    }


def cpu_baseline_large(fa, fb, gamma, w, alphas, slab=1024, n_pix=256, n_planes=4):
    """The oracle, as it stands, on a bounded sample of the large workload,
    extrapolated linearly to the whole job:
      * Gamma of the first ``slab`` detector-A pixels (whole bytes of every
        packed frame) against every detector-B pixel over all N frames; the
        cost is linear in the detector-A pixel count;
      * ``n_pix`` sampled output pixels of ``n_planes`` evenly spaced planes,
        refocused from the device's FP64 Gamma (which the GPU tests show to be
        the exact Gamma of the frames); the cost is linear in the pixel count.
    ``fa``, ``fb``: packed frames on the device; ``gamma``: FP64 view-major
    Gamma on the device."""
    import numpy as np

    import oracle

    threads = _blas_threads()
    n = w.n_frames
    a_slab = fa[:, :slab // 8].cpu().numpy()
    b_all = fb.cpu().numpy()
    t0 = time.perf_counter()
    oracle.correlation(a_slab, b_all, n, slab, w.pb, oracle.FRAMES_BIT1)
    t1 = time.perf_counter()
    del a_slab, b_all
    gam = gamma.cpu().numpy()
    g = oracle.default_geometry(w.wa, w.ha, w.wb, w.hb)
    rng = np.random.default_rng(5)
    ys = rng.integers(0, w.ha, n_pix)
    xs = rng.integers(0, w.wa, n_pix)
    planes = np.unique(np.linspace(0, len(alphas) - 1, n_planes).round().astype(int))
    t2 = time.perf_counter()
    oracle.refocus_pixels(gam, g, np.asarray(alphas)[planes], ys, xs)
    t3 = time.perf_counter()
    del gam
    t_gamma = (t1 - t0) * (w.pa / slab)
    t_plane = (t3 - t2) / planes.size * (w.pa / n_pix)
    return {
        "value": float(n) * w.pa * w.pb / t_gamma,
        "unit": "pixel-pair*frames/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"Gamma of {slab} of {w.pa} detector-A pixels x all {w.pb} detector-B pixels "
                   f"over all {n} frames ({t1 - t0:.2f} s, extrapolated linearly to the whole "
                   f"Gamma: {t_gamma:.0f} s); refocus of {n_pix} output pixels in each of "
                   f"{planes.size} planes ({t3 - t2:.2f} s, extrapolated to {w.pa} pixels per "
                   f"plane: {t_plane:.0f} s per plane)"),
        "extrapolated": True,
        "refocus_planes_per_s": 1.0 / t_plane,
        "seconds": (t1 - t0) + (t3 - t2),
    }


def _layer_level(name):
    return {"enc1": 0, "dec1": 0, "out": 0, "enc2": 1, "dec2": 1, "enc3": 2, "dec3": 2,
            "mid_": 3}[name[:4] if not name.startswith("out") else "out"]


def denoiser_forward_flops(dn, h, w):
    """Algorithmic FLOPs of one forward pass on one h x w plane: two per
    multiply-add of every convolution at its logical channel counts."""
    total = 0
    for L in dn.layers():
        lv = _layer_level(L.name)
        total += 2 * (h >> lv) * (w >> lv) * L.cout_used * L.ks * L.ks * L.cin_used
    return total


def denoiser_train_flops(dn, h, w):
    """One training step per plane: forward, weight gradients, and input
    gradients of every layer but the first."""
    first = dn.layers()[0]
    f0 = 2 * h * w * first.cout_used * first.ks * first.ks * first.cin_used
    return 3 * denoiser_forward_flops(dn, h, w) - f0


def resampled_refocus_bench(cpi, torch, np, dev, g32, geo, w, alphas, reps=3):
    """Refocus with the lens plane sampled at half-pixel steps (2x oversampled,
    (2 Wb - 1) x (2 Hb - 1) samples): the view-resampling kernel against the
    HBM peak (algorithmic bytes: every input view read once, every resampled
    view written once) and the batched refocus over the resampled views."""
    ls = cpi.lens_sampling(2 * w.wb - 1, 2 * w.hb - 1, 0.0, 0.0, 0.5, 0.5)
    gs = cpi.lens_sampling_geometry(geo, ls)
    na = len(alphas)
    ns = ls.nx * ls.ny
    views = torch.empty(ns * w.pa, dtype=torch.float32, device=dev)
    out = torch.empty(na * w.pa, dtype=torch.float32, device=dev)
    ws = cpi.alloc_workspace(cpi.refocus_workspace_size(gs, na), dev)
    cpi.resample_views(g32, geo, ls, views)
    cpi.autotune_refocus(views, gs, alphas, out, workspace=ws)
    torch.cuda.synchronize()
    cpi.profile_begin()
    for _ in range(reps):
        cpi.resample_views(g32, geo, ls, views)
        cpi.refocus(views, gs, alphas, out, workspace=ws)
    torch.cuda.synchronize()
    cpi.profile_end()
    t_res = cpi.profile_query("refocus_resample")[1] / reps
    t_ref = sum(cpi.profile_query(gname)[1] for gname in ("refocus_tables", "refocus_batched")) / reps
    alg = (w.pb + ns) * w.pa * 4
    del views, out, ws
    return {
        "lens_samples": [ls.nx, ls.ny], "step": 0.5, "planes": na,
        "resample_ms": t_res, "refocus_ms": t_ref, "total_ms": t_res + t_ref,
        "resample_roofline": {"bound": "hbm", "achieved": alg / (t_res * 1e-3) / 1e9,
                              "peak": 8000.0, "unit": "GB/s",
                              "frac": alg / (t_res * 1e-3) / 8e12,
                              "algorithmic_bytes": alg},
        "config_kp_rw_splits_kernel_stages": list(cpi.refocus_tiles(gs, na)),
    }


def denoiser_timing(torch, np, dev, batch=16, planes=32, h=128, w=128, reps=100, warmup=10):
    """Training-step and inference time of the denoiser on synthetic planes,
    with the algorithmic BF16 FLOP rate of each against the matrix-core peak."""
    import paper_2407_20692_amd.denoiser as dn

    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    x = torch.randn(planes, h, w, generator=gen, device=dev)
    t = torch.randn(planes, h, w, generator=gen, device=dev)
    net = dn.Denoiser(seed=11, device=dev)
    xb, tb = x[:batch].contiguous(), t[:batch].contiguous()
    out = torch.empty_like(x)
    for _ in range(warmup):
        net.train_step(xb, tb, 1e-4)
        net.forward(x, out=out)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        net.train_step(xb, tb, 1e-4)
    e[1].record()
    e[2].record()
    for _ in range(reps):
        net.forward(x, out=out)
    e[3].record()
    torch.cuda.synchronize()
    ms_step = e[0].elapsed_time(e[1]) / reps
    ms_inf = e[2].elapsed_time(e[3]) / reps
    f_step = denoiser_train_flops(dn, h, w) * batch
    f_inf = denoiser_forward_flops(dn, h, w) * planes
    return {
        "plane": [h, w], "batch": batch, "planes_inferred": planes,
        "train_step_ms": ms_step,
        "train_tflops": f_step / (ms_step * 1e-3) / 1e12,
        "train_frac_bf16_peak": f_step / (ms_step * 1e-3) / BF16_PEAK,
        "inference_ms": ms_inf,
        "inference_tflops": f_inf / (ms_inf * 1e-3) / 1e12,
        "inference_frac_bf16_peak": f_inf / (ms_inf * 1e-3) / BF16_PEAK,
        "flops_note": "algorithmic: 2 per multiply-add at logical channel counts",
    }


def denoise_bench(args, cpi, torch, np, dev):
    """Learned denoiser on pairs made by the pipeline itself, and the
    comparison with the plain pipeline at equal wall time."""
    import paper_2407_20692_amd.denoiser as dn
    import paper_2407_20692_amd.denoise_pipeline as dp
    from synth import WORKLOADS, workload_seed
    from synth.gpu_speckle import generate_binary_frames_gpu

    w = WORKLOADS[DENOISE_WORKLOAD]
    n_few, n_full, na = 500, w.n_frames, w.n_alpha
    geo = cpi.geometry_default(w.wa, w.ha, w.wb, w.hb)
    runs = max(4, args.runs)
    n_test = max(2, runs // 10)
    n_train = runs - n_test
    base = workload_seed(w)

    def frames(r):
        return generate_binary_frames_gpu(w, count=n_full, seed=base + 1000 * r, device=dev,
                                          chunk=2500, mask_seed_value=base + 1000 * r + 7)

    def alphas(r):
        rng = np.random.default_rng(base + 1000 * r + 3)
        return np.sort(rng.uniform(w.alpha_lo, w.alpha_hi, na))

    # -- training pairs -------------------------------------------------------------
    t0 = time.time()
    inputs, targets = dp.make_pairs(frames, alphas, n_train, w.pa, w.pb, geo, n_few, n_full,
                                    log=log)
    torch.cuda.synchronize()
    t_pairs = time.time() - t0
    log(f"denoise: {inputs.shape[0]} training pairs in {t_pairs:.1f} s")

    # -- training ---------------------------------------------------------------------
    net = dn.Denoiser(seed=base, device=dev)
    batch = 16
    # time the training step alone (HIP events), then train
    xb, tb = inputs[:batch].contiguous(), targets[:batch].contiguous()
    for _ in range(3):
        net.train_step(xb, tb, 1e-3)
    net = dn.Denoiser(seed=base, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    reps = 20
    for _ in range(reps):
        net.train_step(xb, tb, 1e-3)
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / reps
    net = dn.Denoiser(seed=base, device=dev)
    t0 = time.time()
    history = dp.train(net, inputs, targets, args.epochs, batch=batch, lr=1e-3, seed=base, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    del inputs, targets

    # -- wall time of the plain pipeline and of inference ---------------------------------
    fa, fb = frames(runs)          # a run used for timing only
    al = alphas(runs)
    out = torch.empty(na, w.ha, w.wa, dtype=torch.float32, device=dev)

    def plain_ms(n, reps=3):
        ts = []
        for _ in range(reps):
            st = cpi.Stream(w.pa, w.pb, cpi.FRAMES_BIT1, 10000)
            ws = cpi.alloc_workspace(cpi.refocus_workspace_size(geo, na), dev)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            pos = 0
            while pos < n:
                k = min(10000, n - pos)
                st.push(fa[pos:pos + k], fb[pos:pos + k], k)
                pos += k
            st.refocus(geo, al, out, workspace=ws)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
            st.close()
        return sorted(ts)[len(ts) // 2]

    ns = [500, 1000, 2000, 5000, 10000, 20000, 50000]
    ts = [plain_ms(n) for n in ns]
    a_ms, b_ms = dp.fit_linear(ns, ts)
    few_planes = torch.empty_like(out)
    dp.prefix_planes(fa, fb, w.pa, w.pb, geo, al, [n_few], [few_planes])
    den = torch.empty_like(out)
    for _ in range(3):
        net.forward(few_planes, out=den)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.forward(few_planes, out=den)
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / 10
    t_budget = ts[0] + t_inf
    n_eq = dp.equal_time_frames(t_budget, a_ms, b_ms, n_few, n_full)
    # acquisition-limited view: frames arrive at the sensor's rate
    rate = 1.0e5
    n_eq_acq = dp.equal_time_frames(n_few / rate * 1e3 + t_budget, a_ms, b_ms + 1e3 / rate,
                                    n_few, n_full)
    del fa, fb

    # -- evaluation on held-out runs -----------------------------------------------------
    res = {"few": [], "den": [], "eq": [], "acq": []}
    for r in range(n_train, runs):
        fa, fb = frames(r)
        al = alphas(r)
        counts = sorted({n_few, n_eq, n_eq_acq, n_full})
        outs = {c: torch.empty(na, w.ha, w.wa, dtype=torch.float32, device=dev) for c in counts}
        dp.prefix_planes(fa, fb, w.pa, w.pb, geo, al, counts, [outs[c] for c in counts])
        tgt = outs[n_full]
        d = dp.denoise_batched(net, outs[n_few])
        for key, pred in (("few", outs[n_few]), ("den", d), ("eq", outs[n_eq]),
                          ("acq", outs[n_eq_acq])):
            p, s, _, _ = dp.quality(pred, tgt)
            res[key].append((p, s))
        del fa, fb
    mean = {k: (float(np.mean([x[0] for x in v])), float(np.mean([x[1] for x in v])))
            for k, v in res.items()}
    pol = dp.decide(mean["den"][0], mean["den"][1], mean["eq"][0], mean["eq"][1], n_few, n_eq)
    pol_acq = dp.decide(mean["den"][0], mean["den"][1], mean["acq"][0], mean["acq"][1], n_few,
                        n_eq_acq)
    fwd = denoiser_forward_flops(dn, w.ha, w.wa)
    step_flops = denoiser_train_flops(dn, w.ha, w.wa) * batch
    return {
        "metric": "denoiser_psnr_ssim_at_equal_time",
        "workload": w.name,
        "n_few": n_few, "n_full": n_full, "planes_per_run": na,
        "train_pairs": n_train * na, "test_pairs": n_test * na, "epochs": args.epochs,
        "batch": batch, "loss_per_epoch": history,
        "seconds": {"pairs": round(t_pairs, 1), "train": round(t_train, 1)},
        "train_step_ms": ms_step,
        "train_tflops": step_flops / (ms_step * 1e-3) / 1e12,
        "train_frac_bf16_peak": step_flops / (ms_step * 1e-3) / BF16_PEAK,
        "inference_ms_32_planes": t_inf,
        "inference_tflops": fwd * na / (t_inf * 1e-3) / 1e12,
        "plain_ms": dict(zip([str(n) for n in ns], ts)),
        "plain_fit_ms": {"a": a_ms, "b_per_frame": b_ms},
        "equal_time": {"budget_ms": t_budget, "n_eq": n_eq},
        "acquisition_limited": {"frames_per_s": rate, "n_eq": n_eq_acq},
        "quality_vs_full": {
            "plain_500": {"psnr": mean["few"][0], "ssim": mean["few"][1]},
            "denoised_500": {"psnr": mean["den"][0], "ssim": mean["den"][1]},
            f"plain_{n_eq}_equal_compute": {"psnr": mean["eq"][0], "ssim": mean["eq"][1]},
            f"plain_{n_eq_acq}_equal_acquisition": {"psnr": mean["acq"][0],
                                                     "ssim": mean["acq"][1]},
        },
        "policy_equal_compute": {"use_denoiser": pol.use_denoiser, "reason": pol.reason},
        "policy_equal_acquisition": {"use_denoiser": pol_acq.use_denoiser,
                                     "reason": pol_acq.reason},
        "dtype": "bf16 matrix cores, fp32 sums and master weights",
        "data": "synthetic",
    }


def refocus_taps(geo, n_alpha):
    """Bilinear taps of a refocus launch: four per (plane, output pixel, view)."""
    return 4 * int(n_alpha) * geo.out_w * geo.out_h * geo.wb * geo.hb


def hot_path(args, cpi, torch, np, dev, w, n, fmt, da, db, alphas, tune=True, plain=True,
             plain_corr=True, plain_planes=None, traffic_key=None):
    """One workload's hot path: the timed step (correlate with Gamma in FP64 and
    FP32, then the batched refocus), per-kernel-group times from the library's
    events on the launch stream, the int8 encoding of the contraction, the
    plain FP32 path and the roofline objects.  Returns (figures, state)."""
    pa, pb = w.pa, w.pb
    gamma = torch.empty(pa * pb, dtype=torch.float64, device=dev)
    g32 = torch.empty(pa * pb, dtype=torch.float32, device=dev)
    # the one-shot workspace, or what memory allows (the library then folds
    # the frames in blocks)
    ws_need = cpi.correlate_workspace_size(n, pa, pb, fmt)
    ws_bytes = min(ws_need, torch.cuda.mem_get_info(dev)[0] - (16 << 30))
    ws_c = cpi.alloc_workspace(ws_bytes, dev)
    geo = cpi.geometry_default(w.wa, w.ha, w.wb, w.hb)
    na = len(alphas)
    out = torch.empty(na * w.pa, dtype=torch.float32, device=dev)
    ws_r = cpi.alloc_workspace(cpi.refocus_workspace_size(geo, na), dev)

    def step():
        cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR,
                      gamma=gamma, gamma_f32=g32, workspace=ws_c)
        cpi.refocus(g32, geo, alphas, out, workspace=ws_r)

    step()
    if tune:
        log(f"bench: autotuning the refocus kernel ({w.name})")
        cpi.autotune_refocus(g32, geo, alphas, out, workspace=ws_r)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps ({w.name})")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    # per-kernel-group times from the library's own events on the launch
    # stream, in a second pass over the same steps (the events add small idle
    # gaps between groups, so they stay out of the timed pass above)
    cpi.profile_begin()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    cpi.profile_end()
    groups = {}
    for grp in ("ingest", "gemm", "refocus_tables", "refocus_batched"):
        cnt, tot = cpi.profile_query(grp)
        groups[grp] = tot / max(cnt, 1)
    ms_corr = groups["ingest"] + groups["gemm"]
    ms_ref = groups["refocus_tables"] + groups["refocus_batched"]

    # the same contraction in the int8 encoding (bit-identical results)
    log("bench: int8 encoding of the contraction")
    cpi.set_mma_encoding(cpi.MMA_INT8)
    try:
        cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR,
                      gamma=gamma, gamma_f32=g32, workspace=ws_c)
        torch.cuda.synchronize()
        reps8 = max(3, args.steps // 4)
        cpi.profile_begin()
        e0.record()
        for _ in range(reps8):
            cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR,
                          gamma=gamma, gamma_f32=g32, workspace=ws_c)
            cpi.refocus(g32, geo, alphas, out, workspace=ws_r)
        e1.record()
        torch.cuda.synchronize()
        cpi.profile_end()
        ms_step_int8 = e0.elapsed_time(e1) / reps8
        cnt, tot = cpi.profile_query("gemm")
        ms_gemm_int8 = tot / max(cnt, 1)
    finally:
        cpi.set_mma_encoding(cpi.MMA_AUTO)

    pairs = float(n) * pa * pb
    fig = {
        "workload": w.name,
        "n_frames": n,
        "correlate_workspace": {"bytes": ws_bytes, "one_shot_bytes": ws_need,
                                "blocked": ws_bytes < ws_need},
        "ms_per_step": ms_step,
        "pixel_pair_frames_per_s": pairs / (ms_step * 1e-3),
        "correlate": {"ms": ms_corr, "ingest_ms": groups["ingest"], "gemm_ms": groups["gemm"],
                      "pixel_pair_frames_per_s": pairs / (ms_corr * 1e-3)},
        "refocus": {"ms": ms_ref, "planes_per_s": na / (ms_ref * 1e-3),
                    "config_kp_rw_splits_kernel_stages": list(cpi.refocus_tiles(geo, na))},
        "int8_step": {"ms_per_step": ms_step_int8,
                      "pixel_pair_frames_per_s": pairs / (ms_step_int8 * 1e-3),
                      "gemm_ms": ms_gemm_int8},
    }

    if plain:
        # plain FP32 comparison path on the same inputs (the one-plane-per-launch
        # refocus on plain_planes of the planes, scaled to the stack)
        log("bench: plain FP32 path")
        al_p = alphas if plain_planes is None else alphas[:plain_planes]
        outp = torch.empty(len(al_p) * w.pa, dtype=torch.float32, device=dev)
        if plain_corr:
            g32p = torch.empty(pa * pb, dtype=torch.float32, device=dev)
            ws_p = cpi.alloc_workspace(cpi.correlate_f32_plain_workspace_size(n, pa, pb, fmt), dev)
            cpi.correlate_f32_plain(da, db, n, pa, pb, fmt, g32p, workspace=ws_p)
        cpi.refocus_plain(g32, geo, al_p, outp, workspace=ws_r)
        torch.cuda.synchronize()
        cpi.profile_begin()
        for _ in range(args.plain_steps):
            if plain_corr:
                cpi.correlate_f32_plain(da, db, n, pa, pb, fmt, g32p, workspace=ws_p)
            cpi.refocus_plain(g32, geo, al_p, outp, workspace=ws_r)
        torch.cuda.synchronize()
        cpi.profile_end()
        pg = {}
        for grp in ("unpack_f32", "sgemm_f32", "refocus_tables", "refocus_plain"):
            cnt, tot = cpi.profile_query(grp)
            pg[grp] = tot / max(cnt, 1)
        ms_corr_p = pg["unpack_f32"] + pg["sgemm_f32"] if plain_corr else float("nan")
        ms_ref_p = (pg["refocus_tables"] + pg["refocus_plain"]) * na / len(al_p)
        if plain_corr:
            del ws_p, g32p
        del outp
        fig["fp32_plain"] = {
            "correlate_ms": ms_corr_p if plain_corr else None,
            "unpack_ms": pg["unpack_f32"] if plain_corr else None,
            "sgemm_ms": pg["sgemm_f32"] if plain_corr else None,
            "pixel_pair_frames_per_s": pairs / (ms_corr_p * 1e-3) if plain_corr else None,
            "sgemm_tflops": 2 * pairs / (pg["sgemm_f32"] * 1e-3) / 1e12 if plain_corr else None,
            "refocus_ms": ms_ref_p, "planes_per_s": na / (ms_ref_p * 1e-3),
            "refocus_planes_timed": len(al_p),
            "mfma_vs_fp32_correlate": ms_corr_p / ms_corr if plain_corr else None,
            "batched_vs_plain_refocus": ms_ref_p / ms_ref,
        }

    gemm_ops = 2.0 * pairs
    achieved = gemm_ops / (groups["gemm"] * 1e-3) / 1e12
    fig["roofline"] = {
        "kernel": "k_gemm_f4lds (FP4 matrix-core contraction, LDS pipeline, exact epilogue)",
        "bound": "mfma",
        "achieved": achieved,
        "peak": FP4_PEAK / 1e12,
        "unit": "TOP/s",
        "frac": achieved * 1e12 / FP4_PEAK,
        # HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (committed
        # summary; None once the kernel source changed)
        "traffic": measured_traffic(pmc_summary("gemm", traffic_key), GEMM_SOURCE),
        "algorithmic_ops_per_launch": gemm_ops,
        "launch_ms": groups["gemm"],
    }
    achieved8 = gemm_ops / (ms_gemm_int8 * 1e-3) / 1e12
    fig["roofline_int8"] = {
        "kernel": "k_gemm_i8lds (int8 matrix-core contraction of bit rows, LDS pipeline, exact epilogue)",
        "bound": "mfma",
        "achieved": achieved8,
        "peak": INT8_PEAK / 1e12,
        "unit": "TOP/s",
        "frac": achieved8 * 1e12 / INT8_PEAK,
        "launch_ms": ms_gemm_int8,
    }
    fig["roofline_refocus"] = refocus_roofline(cpi, geo, alphas, groups["refocus_batched"],
                                               traffic_key)
    # another batched-refocus kernel on the same inputs: for the row-lane
    # kernel, the column-sum kernel's untuned default; otherwise the other of
    # the per-row and column-sum kernels with the same tiles, where it is built
    # for them
    tiles = cpi.refocus_tiles(geo, na)
    if tiles[3] == 2:
        other = (4, 16 if geo.out_h >= 16 else 8, 16, 1, 2)
    else:
        other = (tiles[0], tiles[1], tiles[2], 1 - tiles[3], 2)
    try:
        cpi.refocus_tiled(g32, geo, alphas, out, other, workspace=ws_r)
    except cpi.CpiError:
        other = None
    if other is not None:
        torch.cuda.synchronize()
        cpi.profile_begin()
        for _ in range(max(3, args.steps // 4)):
            cpi.refocus_tiled(g32, geo, alphas, out, other, workspace=ws_r)
        torch.cuda.synchronize()
        cpi.profile_end()
        cnt, tot = cpi.profile_query("refocus_batched")
        fig["roofline_refocus"]["other_kernel"] = {
            "tiles_kp_rw_splits_kernel_stages": list(other), "launch_ms": tot / max(cnt, 1)}
    state = {"gamma": gamma, "g32": g32, "geo": geo, "out": out, "ws_r": ws_r, "ws_c": ws_c}
    return fig, state


def pmc_summary(kind, key):
    """Committed counter summary of a kernel on a workload (None if no key)."""
    if key is None:
        return None
    name = {"gemm": f"gemm_f4lds_{key[0]}_pmc.txt", "refocus": f"ref_sep_{key[1]}_pmc.txt",
            "refocus_rows": f"ref_rows_{key[1]}_pmc.txt"}[kind]
    return os.path.join(ROOT, "profiles", name)


def refocus_roofline(cpi, geo, alphas, launch_ms, traffic_key):
    """The batched refocus kernel against the vector-ALU roof: two FLOPs (one
    multiply-add) per bilinear tap, four taps per (plane, output pixel, view).
    Beside it: the measured HBM traffic (counters) and the per-plane footprint
    bytes (every Gamma element a plane's samples touch, counted exactly), which
    exceed what HBM moves because the planes of a work-group share each staged
    view window."""
    na = len(alphas)
    taps = refocus_taps(geo, na)
    flops = 2.0 * taps
    achieved = flops / (launch_ms * 1e-3) / 1e12
    tiles = cpi.refocus_tiles(geo, na)
    foot = refocus_algorithmic_bytes(geo, alphas)
    rows = tiles[3] == 2
    summary = pmc_summary("refocus_rows" if rows else "refocus", traffic_key)
    source = ROWS_SOURCE if rows else REF_SOURCE
    traffic = measured_traffic(summary, source, tiles)
    r = {
        "kernel": ("k_ref_rows + k_ref_rows_fold (row-lane x pass: lanes are view rows, window "
                   "staged column by column in LDS, column cells and weights from a per-view "
                   "table; then the fold over y_b)" if rows else
                   "k_ref_sep (planes batched per work-group, LDS-staged view windows, column "
                   "interpolants summed over x_b before the row weights)" if tiles[3] == 1 else
                   "k_ref_batched (planes batched per work-group, LDS-staged view windows)"),
        "tiles_kp_rw_splits_kernel_stages": list(tiles),
        "bound": "alu",
        "achieved": achieved,
        "peak": FP32_VECTOR_PEAK / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved * 1e12 / FP32_VECTOR_PEAK,
        "frac_of_unpacked_fp32": achieved * 1e12 / FP32_UNPACKED_PEAK,
        "algorithmic_flops_per_launch": flops,
        "taps_per_launch": taps,
        "launch_ms": launch_ms,
        "traffic": traffic,
        "footprint_bytes_per_launch": foot,
        "footprint_GBps": foot / (launch_ms * 1e-3) / 1e9,
    }
    if traffic:
        bw = traffic / (launch_ms * 1e-3) / 1e9
        r["hbm"] = {"GBps": bw, "peak": 8000.0, "frac": bw / 8000.0}
    lds = measured_lds(summary, source, tiles)
    if lds:
        bw = lds / (launch_ms * 1e-3) / 1e12
        r["lds"] = {"bytes_per_launch": lds, "TBps": bw, "peak": LDS_PEAK / 1e12,
                    "frac": bw * 1e12 / LDS_PEAK,
                    "note": "LDS bytes read per launch from rocprofv3 counters (committed "
                            "summary taken on this kernel source and tiles) over the whole "
                            "refocus call's time"}
    return r


def streaming_bench(args, cpi, torch, np, dev):
    """The streamed workload: 1000-frame 1-bit chunks (Da 128x128, Db 64x64),
    all distinct (made on the device, staged in pinned host memory), each
    pushed from the host and followed by a 32-plane refocus.  Overlapped: the
    handle keeps two FP32 Gamma buffers and the refocus of chunk k runs on a
    second stream while chunk k + 1 is copied and folded; serial: both on one
    stream.  All chunks are enqueued without host waits; latency per chunk is
    the device time from the start of its copy to the end of its refocus
    (events), sustained frames/s the whole run's wall time."""
    from synth import WORKLOADS, alphas_for
    from synth.gpu_speckle import generate_binary_frames_gpu

    ws = WORKLOADS[STREAM_WORKLOAD]
    chunks = min(args.stream_chunks, ws.n_frames // ws.chunk)
    log(f"bench: streaming {chunks} distinct chunks of {ws.chunk}")
    fa, fb = generate_binary_frames_gpu(ws, count=chunks * ws.chunk, device=dev)
    ca = fa.cpu().pin_memory()
    cb = fb.cpu().pin_memory()
    # one device copy of every pinned chunk before timing: the first DMA over
    # a pinned page pays a one-time mapping cost (measured: up to 17 ms of
    # host stall in the first timed pass otherwise)
    fa.copy_(ca)
    fb.copy_(cb)
    torch.cuda.synchronize()
    del fa, fb
    sgeo = cpi.geometry_default(ws.wa, ws.ha, ws.wb, ws.hb)
    sal = alphas_for(ws)
    sout = torch.empty(len(sal) * ws.pa, dtype=torch.float32, device=dev)
    sws = cpi.alloc_workspace(cpi.refocus_workspace_size(sgeo, len(sal)), dev)

    su_, sr_ = torch.cuda.Stream(), torch.cuda.Stream()   # the same two for both runs

    def run(overlap):
        su = su_
        sr = sr_ if overlap else su
        nbuf = 2 if overlap else 1

        def chunk(st, k):
            st.push_host(ca[k * ws.chunk:(k + 1) * ws.chunk].reshape(-1),
                         cb[k * ws.chunk:(k + 1) * ws.chunk].reshape(-1), ws.chunk)
            if overlap:
                st.refocus_async(sgeo, sal, sout, sws, sr)
            else:
                st.refocus(sgeo, sal, sout, workspace=sws)

        # warm-up on a separate stream object: one untimed pass over all the
        # chunks (kernels loaded, tables cached; the host copies of a
        # process's first fraction of a second of streaming stalled the host
        # for up to 20 ms at times)
        warm = cpi.Stream(ws.pa, ws.pb, cpi.FRAMES_BIT1, max_chunk=ws.chunk, device=dev,
                          stream=su, gamma_buffers=nbuf)
        for k in range(chunks):
            chunk(warm, k)
        torch.cuda.synchronize()
        warm.close()
        st = cpi.Stream(ws.pa, ws.pb, cpi.FRAMES_BIT1, max_chunk=ws.chunk, device=dev,
                        stream=su, gamma_buffers=nbuf)
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(chunks)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(chunks)]
        # (torch makes a HIP event at its first record: done here, outside the
        # timed loop, where 400 fresh events stalled the first timed pass)
        for e in ev0 + ev1:
            e.record(su)
        torch.cuda.synchronize()
        gc.disable()   # no collector pauses between the enqueues
        try:
            t_start = time.perf_counter()
            for k in range(chunks):
                ev0[k].record(su)
                chunk(st, k)
                ev1[k].record(sr)
            torch.cuda.synchronize()
            t_total = time.perf_counter() - t_start
        finally:
            gc.enable()
        lat = [ev0[k].elapsed_time(ev1[k]) for k in range(chunks)]
        res = {
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "frames_per_s": chunks * ws.chunk / t_total,
            "device_frames_per_s": chunks * ws.chunk / (ev0[0].elapsed_time(ev1[-1]) * 1e-3),
            "final_frames": st.frames,
        }
        st.close()
        return res

    log("bench: streaming, update and refocus on one stream")
    one = run(False)
    log("bench: streaming, refocus on a second stream")
    two = run(True)
    res = {
        "workload": ws.name,
        "chunks": chunks,
        "chunk_frames": ws.chunk,
        "frames": f"{chunks} distinct seeded chunks ({chunks * ws.chunk} frames, made on the "
                  f"device, pushed from pinned host memory)",
        "mode": "update and refocus of each chunk on one stream; the host copy of chunk k + 1 "
                "runs on the library's copy stream during the work on chunk k; latency = device "
                "time from a chunk's copy to the end of its refocus",
        "n_alpha": len(sal),
    }
    res.update(one)
    two["mode"] = ("refocus of chunk k on a second stream while chunk k + 1 is folded (two FP32 "
                   "Gamma buffers); the two streams' kernels share the CUs, and the gain depends "
                   "on how the runtime places the streams on its hardware queues (1.1-1.33e6 "
                   "frames/s measured over runs)")
    res["two_stream_refocus"] = two
    return res


# the denoiser figures when main() took them first
_DENOISER_TIMING = []


def next_rows(cpi, torch, np, dev, g32, geo, w, alphas):
    """NEXT rows measured on the paper-like Gamma: the paper's stack sizes,
    the resampled lens plane, raw-file ingest and the denoiser's kernels."""
    counts = {}
    for na in (100, 261, 1000):
        al = np.linspace(0.5, 1.5, na)
        o = torch.empty(na * w.pa, dtype=torch.float32, device=dev)
        ws_n = cpi.alloc_workspace(cpi.refocus_workspace_size(geo, na), dev)
        cpi.autotune_refocus(g32, geo, al, o, workspace=ws_n)
        torch.cuda.synchronize()
        cpi.profile_begin()
        for _ in range(3):
            cpi.refocus(g32, geo, al, o, workspace=ws_n)
        torch.cuda.synchronize()
        cpi.profile_end()
        t = sum(cpi.profile_query(gname)[1] for gname in ("refocus_tables", "refocus_batched")) / 3
        counts[str(na)] = {"ms": t, "planes_per_s": na / (t * 1e-3),
                           "config_kp_rw_splits_kernel_stages": list(cpi.refocus_tiles(geo, na))}
        del o, ws_n
    res = {"refocus_plane_counts": counts}
    res["refocus_resampled"] = resampled_refocus_bench(cpi, torch, np, dev, g32, geo, w, alphas)
    res["file_ingest"] = file_ingest_bench(cpi, torch, np, dev)
    if _DENOISER_TIMING:
        res["denoiser"] = _DENOISER_TIMING[0]
    else:
        log("bench: denoiser training step and inference")
        res["denoiser"] = denoiser_timing(torch, np, dev)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 3 for the paper workload)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 3; 1 for the paper workload)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--stream-chunks", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 path")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the paper-like sub-line, plane counts, resampled lens plane, "
                         "raw-file ingest and denoiser measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", choices=["large", "paper_like", "paper", "denoise",
                                           "denoise_step"],
                    default="large",
                    help="large (default line): Da 256x256, Db 128x128, N=100000 distinct "
                         "packed-bit frames, 128 planes, with the paper-like workload and the "
                         "streamed workload as sub-objects; paper_like: Da 128x128, Db 64x64, "
                         "N=20000 bytes, 32 planes; paper: 256x256 on both detectors, --files "
                         "files of 512 frames, 261 planes (the paper's benchmark configuration); "
                         "denoise: train the learned denoiser on pipeline-made pairs "
                         "(500 -> 50000 frames) and compare with the plain pipeline at "
                         "equal wall time; denoise_step: time the denoiser's training "
                         "step and inference only")
    ap.add_argument("--runs", type=int, default=625,
                    help="denoise workload: streams of 50000 frames (32 pairs each)")
    ap.add_argument("--epochs", type=int, default=4, help="denoise workload: training epochs")
    ap.add_argument("--files", type=int, default=7808,
                    help="paper workload: files of 512 frames (the paper uses 11, 100, 500, 7808)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 3 if args.workload == "paper" else 20
    if args.warmup is None:
        args.warmup = 1 if args.workload == "paper" else 3
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 5}))
        return

    import paper_2407_20692_amd as cpi
    from synth import WORKLOADS, alphas_for, generate_frames

    if args.workload == "denoise":
        print(json.dumps(denoise_bench(args, cpi, torch, np, dev)))
        return
    if args.workload == "denoise_step":
        print(json.dumps(denoiser_timing(torch, np, dev)))
        return

    paper = args.workload == "paper"
    large = args.workload == "large"
    if not args.no_next and not paper:
        # timed before the other parts make their streams: the training step
        # runs on three streams, and with more streams than the runtime's
        # hardware queues (four by default) they start sharing queues
        log("bench: denoiser training step and inference")
        _DENOISER_TIMING.append(denoiser_timing(torch, np, dev))
    w = WORKLOADS[PAPER_WORKLOAD if paper else (LARGE_WORKLOAD if large else WORKLOAD)]
    log(f"bench: generating {w.name}")
    alphas = alphas_for(w)
    n, pa, pb = w.n_frames, w.pa, w.pb
    a = b = None
    if paper:
        n = args.files * 512
    if large or paper:
        from synth.gpu_speckle import generate_binary_frames_gpu
        fmt = cpi.FRAMES_BIT1
        fa, fb = generate_binary_frames_gpu(w, count=n, device=dev)
        da, db = fa.reshape(-1), fb.reshape(-1)
        frames_desc = f"1-bit packed, frame-major, {n} distinct frames generated on the device"
    else:
        fmt = cpi.FRAMES_U8
        a, b = generate_frames(w)
        da = torch.from_numpy(a.reshape(-1)).to(dev)
        db = torch.from_numpy(b.reshape(-1)).to(dev)
        frames_desc = "uint8 0/1, frame-major"
    name = w.name if not paper else f"{w.name.split('_files')[0]}_files{args.files}_bit1"
    # (the paper workload keeps the default refocus configuration: each timed
    # candidate would take about a second at its size; its plain FP32
    # correlator runs up to 51200 frames, whose FP32 copies fit)
    fig, state = hot_path(args, cpi, torch, np, dev, w, n, fmt, da, db, alphas,
                          tune=not paper, plain=not args.no_plain,
                          plain_corr=not (paper and n > 51200),
                          plain_planes=(4 if paper else (8 if large else None)),
                          traffic_key=(LARGE_KEY if large else (PAPER_LIKE_KEY if not paper
                                                                else None)))
    pairs = float(n) * pa * pb
    line = {
        "metric": "\u0393 pixel-pair\u00b7frames/s and refocused planes/s: int8-MFMA vs plain FP32, 1 GPU",
        "value": pairs / (fig["ms_per_step"] * 1e-3),
        "unit": "pixel-pair*frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fig["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4-e2m1 0/1 operands, fp32 sums (exact); int64/fp64 epilogue; fp32 refocus",
        "data": "synthetic",
        "config": {"workload": name, "n_frames": n, "pa": pa, "pb": pb, "frames": frames_desc,
                   "n_alpha": len(alphas),
                   "alpha_range": [float(alphas[0]), float(alphas[-1])],
                   "gamma_outputs": "FP64 + FP32, view-major",
                   "contraction_encoding": ("FP4 (E2M1) 0/1 operands on the FP4 matrix cores "
                                            "(exact); the int8 encoding of the same step is in "
                                            "int8_step and roofline_int8")},
    }
    for k in ("correlate", "refocus", "int8_step", "fp32_plain", "roofline", "roofline_int8",
              "roofline_refocus"):
        if k in fig:
            line[k] = fig[k]
    line["int8_step"]["vs_fp32_plain_correlate"] = (
        fig["fp32_plain"]["correlate_ms"] / fig["int8_step"]["gemm_ms"]
        if fig.get("fp32_plain", {}).get("correlate_ms") else None)

    if large and not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (sample of the large workload)")
        line["cpu_baseline"] = cpu_baseline_large(fa, fb, state["gamma"], w, alphas)
    if large or paper:
        del da, db, fa, fb, state
        torch.cuda.empty_cache()

    if large and not args.no_next:
        # the paper-like workload as a sub-object (its own steps and rooflines)
        wl = WORKLOADS[WORKLOAD]
        log(f"bench: generating {wl.name}")
        al2 = alphas_for(wl)
        a2, b2 = generate_frames(wl)
        da2 = torch.from_numpy(a2.reshape(-1)).to(dev)
        db2 = torch.from_numpy(b2.reshape(-1)).to(dev)
        fig2, st2 = hot_path(args, cpi, torch, np, dev, wl, wl.n_frames, cpi.FRAMES_U8, da2, db2,
                             al2, tune=True, plain=not args.no_plain, traffic_key=PAPER_LIKE_KEY)
        line["paper_like"] = fig2
        line.update(next_rows(cpi, torch, np, dev, st2["g32"], st2["geo"], wl, al2))
        del da2, db2, st2
    elif args.workload == "paper_like" and not args.no_next:
        line.update(next_rows(cpi, torch, np, dev, state["g32"], state["geo"], w, alphas))

    if not args.no_stream and not paper:
        line["streaming"] = streaming_bench(args, cpi, torch, np, dev)

    # the device's own sustained figures beside the vendor peaks
    mp = cpi.measure_peaks(dev)
    line["measured_peaks"] = {
        "int8_TOPs": mp["int8_ops_per_s"] / 1e12, "fp4_TOPs": mp["fp4_ops_per_s"] / 1e12,
        "copy_GBps": mp["copy_bytes_per_s"] / 1e9,
        "vendor": {"int8_TOPs": INT8_PEAK / 1e12, "fp4_TOPs": FP4_PEAK / 1e12, "hbm_GBps": 8000.0},
        "what": "register-only loops of the two matrix-core ops on binary-like operands; "
                "1 GiB device copy, read + write bytes",
    }
    line["roofline"]["frac_of_measured_peak"] = (line["roofline"]["achieved"] * 1e12
                                                 / mp["fp4_ops_per_s"])
    line["roofline_int8"]["frac_of_measured_peak"] = (line["roofline_int8"]["achieved"] * 1e12
                                                      / mp["int8_ops_per_s"])

    if args.workload == "paper_like" and not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(a, b, w, alphas)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
