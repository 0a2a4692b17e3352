#!/usr/bin/env python3
"""Benchmark of the correlation plenoptic imaging hot path on one MI355X.

Workload: Da 128x128, Db 64x64, N = 20000 binary frames stored as bytes
(SPAD-like occupancy ~0.1, seeded speckle through a 3-slit mask), 32 refocus
planes alpha in [0.5, 1.5].  One step is one pass of the hot path with the
inputs resident in HBM: ingest + matrix-core contraction with the exact
int64/FP64 epilogue (Gamma in FP64 and FP32) + batched refocus of 32 planes
with the autotuned configuration (tuned once before timing).  Binary frames
are contracted as FP4 (E2M1) 0/1 operands with FP32 sums, exact below 2^24
frames per pass; the int8 encoding of the same contraction is timed beside it.

Printed as ONE JSON line:
  value          Gamma pixel-pair*frames per second over the whole step
                 (N * Pa * Pb per step / step time)
  refocus        refocused planes per second of the batched kernel
  fp32_plain     the plain FP32 path on the same inputs (correlator and
                 one-plane-per-launch refocus) and the int8/FP32 ratios
  streaming      chunk-to-stack latency p50/p99 and frames/s for 1000-frame
                 1-bit chunks of the same geometry, each followed by a
                 32-plane refocus
  roofline       the contraction kernel (dominant) against the FP4 peak,
                 its duration measured with HIP events on its stream
  roofline_int8  the same contraction in the int8 encoding against the int8 peak
  roofline_refocus  the batched refocus kernel: algorithmic (footprint) bytes
                 per launch over its duration, against the HBM peak
  refocus_plane_counts  the paper's stack sizes (100, 261, 1000 planes)
  file_ingest    raw side-by-side frame files (the paper's 256 x 512 layout,
                 11 files of 512 frames) streamed into the running sums
  measured_peaks the device's sustained matrix-core and copy rates (microbenchmarks)
  refocus_resampled  refocusing with the lens plane sampled at half-pixel steps
                 (general 4-D multilinear interpolation): view resampling + refocus
  denoiser       the learned denoiser's training step (16 planes of 128 x 128)
                 and inference (32 planes): time and algorithmic BF16 FLOP rate
  cpu_baseline   the CPU oracle on a bounded sample of the same workload
"""
import argparse
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
PMC_SUMMARY = os.path.join(ROOT, "profiles", "gemm_f4lds_da128_db64_n20000_pmc.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_2407_20692_amd", "csrc", "kernels_gemm.hip")
REF_PMC_SUMMARY = os.path.join(ROOT, "profiles", "ref_sep_da128_db64_32planes_pmc.txt")
REF_SOURCE = os.path.join(ROOT, "paper_2407_20692_amd", "csrc", "kernels_refocus.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(summary=None, source=None, tiles=None):
    """HBM bytes per launch from a committed counter summary (the contraction's
    by default), if it was taken on the current kernel source (and, for the
    refocus, with these tiles); else None."""
    summary = summary or PMC_SUMMARY
    source = source or GEMM_SOURCE
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
    key = "hbm_bytes_per_launch"
    if tiles is not None:
        key = "hbm_bytes_per_launch_tiles " + " ".join(str(int(v)) for v in tiles)
    try:
        return float(fields[key].split()[0])
    except (KeyError, ValueError, IndexError):
        return None


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


def cpu_baseline(a, b, w, alphas):
    """The oracle, as it stands, on a bounded sample of the workload (about
    12 s of host work): Gamma for every pixel pair over all frames, and 10 of
    the refocus planes (evenly spaced, first and last included)."""
    import numpy as np

    import oracle

    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
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


def denoiser_timing(torch, np, dev, batch=16, planes=32, h=128, w=128, reps=20):
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
    for _ in range(3):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--stream-chunks", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the plane-count refocus and raw-file ingest measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", choices=["paper_like", "large", "paper", "denoise",
                                           "denoise_step"],
                    default="paper_like",
                    help="paper_like: Da 128x128, Db 64x64, N=20000 bytes (default line); "
                         "large: Da 256x256, Db 128x128, N=100000 packed bits, 128 planes; "
                         "paper: 256x256 on both detectors, --files files of 512 frames, "
                         "261 planes (the paper's benchmark configuration); "
                         "denoise: train the learned denoiser on pipeline-made pairs "
                         "(500 -> 50000 frames) and compare with the plain pipeline at "
                         "equal wall time; denoise_step: time the denoiser's training "
                         "step and inference only")
    ap.add_argument("--runs", type=int, default=625,
                    help="denoise workload: streams of 50000 frames (32 pairs each)")
    ap.add_argument("--epochs", type=int, default=4, help="denoise workload: training epochs")
    ap.add_argument("--files", type=int, default=11,
                    help="paper workload: files of 512 frames (the paper uses 11, 100, 500, 7808)")
    args = ap.parse_args()
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
    from synth import WORKLOADS, alphas_for, generate_frames, pack_bits_lsb

    if args.workload == "denoise":
        print(json.dumps(denoise_bench(args, cpi, torch, np, dev)))
        return
    if args.workload == "denoise_step":
        print(json.dumps(denoiser_timing(torch, np, dev)))
        return

    paper = args.workload == "paper"
    large = args.workload == "large" or paper
    w = WORKLOADS[PAPER_WORKLOAD if paper else (LARGE_WORKLOAD if large else WORKLOAD)]
    log(f"bench: generating {w.name}")
    alphas = alphas_for(w)
    n, pa, pb = w.n_frames, w.pa, w.pb
    generated = None
    if paper:
        n = args.files * 512
    if large:
        from synth.gpu_speckle import generate_binary_frames_gpu
        fmt = cpi.FRAMES_BIT1
        base = min(n, 25600)
        pa_bits, pb_bits = generate_binary_frames_gpu(w, count=base, device=dev)
        if base < n:
            # more frames than generated: the generated block repeats (the
            # contraction's work does not depend on the frame contents)
            def tiled(x):
                t = torch.empty((n, x.shape[1]), dtype=x.dtype, device=dev)
                for lo in range(0, n, base):
                    t[lo:lo + base] = x[:min(base, n - lo)]
                return t
            pa_bits, pb_bits = tiled(pa_bits), tiled(pb_bits)
            generated = base
        da, db = pa_bits.reshape(-1), pb_bits.reshape(-1)
        a = b = None
    else:
        fmt = cpi.FRAMES_U8
        a, b = generate_frames(w)
        da = torch.from_numpy(a.reshape(-1)).to(dev)
        db = torch.from_numpy(b.reshape(-1)).to(dev)
    gamma = torch.empty(pa * pb, dtype=torch.float64, device=dev)
    g32 = torch.empty(pa * pb, dtype=torch.float32, device=dev)
    ws_c = cpi.alloc_workspace(cpi.correlate_workspace_size(n, pa, pb, fmt), dev)
    geo = cpi.geometry_default(w.wa, w.ha, w.wb, w.hb)
    out = torch.empty(len(alphas) * w.pa, dtype=torch.float32, device=dev)
    ws_r = cpi.alloc_workspace(cpi.refocus_workspace_size(geo, len(alphas)), dev)

    def step():
        cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR,
                      gamma=gamma, gamma_f32=g32, workspace=ws_c)
        cpi.refocus(g32, geo, alphas, out, workspace=ws_r)

    step()
    if not paper:
        # (the paper workload keeps the default configuration: each timed
        # candidate would take about a second at its size)
        log("bench: autotuning the refocus kernel")
        cpi.autotune_refocus(g32, geo, alphas, out, workspace=ws_r)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
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
        cpi.profile_begin()
        for _ in range(max(3, args.steps // 4)):
            cpi.correlate(da, db, n, pa, pb, fmt, cpi.GAMMA_VIEW_MAJOR,
                          gamma=gamma, gamma_f32=g32, workspace=ws_c)
        torch.cuda.synchronize()
        cpi.profile_end()
        cnt, tot = cpi.profile_query("gemm")
        ms_gemm_int8 = tot / max(cnt, 1)
    finally:
        cpi.set_mma_encoding(cpi.MMA_AUTO)

    # plain FP32 comparison path on the same inputs (at the paper workload's
    # size: the correlator up to 51200 frames, whose FP32 copies of the frames
    # fit, and the one-plane-per-launch refocus on 4 of the planes)
    log("bench: plain FP32 path")
    plain_corr = not (paper and n > 51200)
    al_p = alphas[:4] if paper else alphas
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
    # plain refocus time per call scaled to the full stack
    ms_ref_p = (pg["refocus_tables"] + pg["refocus_plain"]) * len(alphas) / len(al_p)
    if plain_corr:
        del ws_p, g32p
    del outp

    pairs = float(n) * pa * pb
    line = {
        "metric": "Gamma pixel-pair*frames/s and refocused planes/s: int8-MFMA vs plain FP32, 1 GPU",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pixel-pair*frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4-e2m1 0/1 operands, fp32 sums (exact); int64/fp64 epilogue; fp32 refocus",
        "data": "synthetic",
        "config": {"workload": w.name if not paper else f"{w.name.split('_files')[0]}_files{args.files}_bit1",
                   "n_frames": n, "pa": pa, "pb": pb,
                   "frames": ("1-bit packed, frame-major (generated on the device"
                              + (f"; {generated} distinct frames, repeated)" if generated else ")")
                              if large else "uint8 0/1, frame-major"), "n_alpha": len(alphas),
                   "alpha_range": [float(alphas[0]), float(alphas[-1])],
                   "gamma_outputs": "FP64 + FP32, view-major"},
        "correlate": {"ms": ms_corr, "ingest_ms": groups["ingest"], "gemm_ms": groups["gemm"],
                      "pixel_pair_frames_per_s": pairs / (ms_corr * 1e-3)},
        "refocus": {"ms": ms_ref, "planes_per_s": len(alphas) / (ms_ref * 1e-3),
                    "config_kp_rw_splits_kernel_stages": list(cpi.refocus_tiles(geo, len(alphas)))},
        "fp32_plain": {
            "correlate_ms": ms_corr_p if plain_corr else None,
            "unpack_ms": pg["unpack_f32"] if plain_corr else None,
            "sgemm_ms": pg["sgemm_f32"] if plain_corr else None,
            "pixel_pair_frames_per_s": pairs / (ms_corr_p * 1e-3) if plain_corr else None,
            "sgemm_tflops": 2 * pairs / (pg["sgemm_f32"] * 1e-3) / 1e12 if plain_corr else None,
            "refocus_ms": ms_ref_p, "planes_per_s": len(alphas) / (ms_ref_p * 1e-3),
            "refocus_planes_timed": len(al_p),
            "mfma_vs_fp32_correlate": ms_corr_p / ms_corr if plain_corr else None,
            "batched_vs_plain_refocus": ms_ref_p / ms_ref,
        },
    }

    gemm_ops = 2.0 * pairs
    achieved = gemm_ops / (groups["gemm"] * 1e-3) / 1e12
    line["roofline"] = {
        "kernel": "k_gemm_f4lds (FP4 matrix-core contraction, LDS pipeline, exact epilogue)",
        "bound": "mfma",
        "achieved": achieved,
        "peak": FP4_PEAK / 1e12,
        "unit": "TOP/s",
        "frac": achieved * 1e12 / FP4_PEAK,
        "traffic": measured_traffic(),
        "algorithmic_ops_per_launch": gemm_ops,
        "launch_ms": groups["gemm"],
    }
    ref_bytes = refocus_algorithmic_bytes(geo, alphas)
    ref_bw = ref_bytes / (groups["refocus_batched"] * 1e-3) / 1e9
    tiles = cpi.refocus_tiles(geo, len(alphas))
    line["roofline_refocus"] = {
        "kernel": ("k_ref_sep (planes batched per work-group, LDS-staged view windows, column "
                   "interpolants summed over x_b before the row weights)" if tiles[3] == 1 else
                   "k_ref_batched (planes batched per work-group, LDS-staged view windows)"),
        "tiles_kp_rw_splits_kernel_stages": list(tiles),
        "bound": "hbm",
        "achieved": ref_bw,
        "peak": 8000.0,
        "unit": "GB/s",
        "frac": ref_bw / 8000.0,
        "algorithmic_bytes_per_launch": ref_bytes,
        "launch_ms": groups["refocus_batched"],
        # HBM bytes per launch of the tuned column-sum kernel from rocprofv3
        # FETCH_SIZE / WRITE_SIZE (committed summary; None once the source
        # changed or the tuned tiles differ from the profiled ones)
        "traffic": measured_traffic(REF_PMC_SUMMARY, REF_SOURCE, tiles),
        "note": "achieved = footprint bytes of every plane (counted exactly) / launch time; planes "
                "share each staged view window, so this exceeds what HBM moves (traffic, from "
                "rocprofv3 counters) and the kernel is bound by LDS reads and per-view latency "
                "rather than HBM",
    }
    # the other batched-refocus kernel with the same tiles (same inputs), where
    # it is built for them (the column-sum kernel also takes shapes the
    # per-row kernel does not)
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
        line["roofline_refocus"]["other_kernel_same_tiles"] = {
            "tiles_kp_rw_splits_kernel_stages": list(other), "launch_ms": tot / max(cnt, 1)}
    achieved8 = gemm_ops / (ms_gemm_int8 * 1e-3) / 1e12
    line["roofline_int8"] = {
        "kernel": "k_gemm<bits> (int8 matrix-core contraction, exact epilogue)",
        "bound": "mfma",
        "achieved": achieved8,
        "peak": INT8_PEAK / 1e12,
        "unit": "TOP/s",
        "frac": achieved8 * 1e12 / INT8_PEAK,
        "launch_ms": ms_gemm_int8,
    }

    if large or paper:
        # counters were taken on the paper-like workload
        line["roofline"]["traffic"] = None
        line["roofline_refocus"]["traffic"] = None
    rt = line["roofline_refocus"]["traffic"]
    if rt:
        # what the measured HBM traffic amounts to at this launch time
        bw = rt / (groups["refocus_batched"] * 1e-3) / 1e9
        line["roofline_refocus"]["traffic_GBps"] = bw
        line["roofline_refocus"]["traffic_frac"] = bw / 8000.0
    if not args.no_stream and not large:
        ws = WORKLOADS[STREAM_WORKLOAD]
        log(f"bench: streaming {args.stream_chunks} chunks of {ws.chunk}")
        distinct = 20
        sa_, sb_ = generate_frames(ws, count=distinct * ws.chunk)
        ca = torch.from_numpy(pack_bits_lsb(sa_)).pin_memory()
        cb = torch.from_numpy(pack_bits_lsb(sb_)).pin_memory()
        fa_b, fb_b = cpi.frame_bytes(ws.pa, cpi.FRAMES_BIT1), cpi.frame_bytes(ws.pb, cpi.FRAMES_BIT1)
        st = cpi.Stream(ws.pa, ws.pb, cpi.FRAMES_BIT1, max_chunk=ws.chunk, device=dev)
        sgeo = cpi.geometry_default(ws.wa, ws.ha, ws.wb, ws.hb)
        sal = alphas_for(ws)
        sout = torch.empty(len(sal) * ws.pa, dtype=torch.float32, device=dev)
        sws = cpi.alloc_workspace(cpi.refocus_workspace_size(sgeo, len(sal)), dev)
        lat = []
        dev_lat = []
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.stream_chunks):
            j = k % distinct
            cha = ca.view(-1, fa_b)[j * ws.chunk:(j + 1) * ws.chunk].reshape(-1)
            chb = cb.view(-1, fb_b)[j * ws.chunk:(j + 1) * ws.chunk].reshape(-1)
            t0 = time.perf_counter()
            ev0.record()
            st.push_host(cha, chb, ws.chunk)
            st.refocus(sgeo, sal, sout, workspace=sws)
            ev1.record()
            ev1.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            dev_lat.append(ev0.elapsed_time(ev1))
        t_total = time.perf_counter() - t_start
        line["streaming"] = {
            "workload": ws.name,
            "chunks": args.stream_chunks,
            "chunk_frames": ws.chunk,
            "frames": f"first {distinct} seeded chunks of the workload, cycled",
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "device_p50_ms": float(np.percentile(dev_lat, 50)),
            "device_p99_ms": float(np.percentile(dev_lat, 99)),
            "frames_per_s": args.stream_chunks * ws.chunk / t_total,
            "n_alpha": len(sal),
        }
        st.close()

    # the device's own sustained figures beside the vendor peaks
    mp = cpi.measure_peaks(dev)
    line["measured_peaks"] = {
        "int8_TOPs": mp["int8_ops_per_s"] / 1e12, "fp4_TOPs": mp["fp4_ops_per_s"] / 1e12,
        "copy_GBps": mp["copy_bytes_per_s"] / 1e9,
        "vendor": {"int8_TOPs": INT8_PEAK / 1e12, "fp4_TOPs": FP4_PEAK / 1e12, "hbm_GBps": 8000.0},
        "what": "register-only loops of the two matrix-core ops on binary-like operands; "
                "1 GiB device copy, read + write bytes",
    }
    line["roofline"]["frac_of_measured_peak"] = achieved * 1e12 / mp["fp4_ops_per_s"]
    line["roofline_int8"]["frac_of_measured_peak"] = achieved8 * 1e12 / mp["int8_ops_per_s"]

    if not args.no_next and not large:
        # the paper's stack sizes (100, 261, 1000 planes) on the same Gamma
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
        line["refocus_plane_counts"] = counts
        line["refocus_resampled"] = resampled_refocus_bench(cpi, torch, np, dev, g32, geo, w,
                                                            alphas)
        line["file_ingest"] = file_ingest_bench(cpi, torch, np, dev)
        log("bench: denoiser training step and inference")
        line["denoiser"] = denoiser_timing(torch, np, dev)

    if not args.no_cpu_baseline and not large:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(a, b, w, alphas)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
