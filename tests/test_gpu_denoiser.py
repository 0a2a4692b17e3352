"""GPU parity of the learned denoiser's kernels and network against the FP64
oracle (``oracle.denoiser``), called through the C ABI.

Tolerances follow from the arithmetic.  Inputs and weights are bfloat16
values on both sides, so every product is exact in FP32; a sum of K terms in
FP32 is within K * 2^-23 * S of the exact sum (S = sum of |terms|, the factor
2 over the round-to-nearest bound covering truncating accumulation), and a
stored bfloat16 result adds at most 2^-9 |value| (2^-8 is used).  Routing
kernels (pooling, upsampling, concatenation) are bit-exact.  End to end, both
sides round at the same points, so they differ only where an FP32 sum and an
FP64 sum round to different bfloat16 neighbours, and those one-ulp
differences propagate through 15 layers.  Injecting noise of the size of FP32
accumulation error (sqrt(K) * 2^-24 * S) before every rounding of the FP64
oracle moves its output by 0.7% of max |f(x)| and its per-layer weight
gradients by 0.1% (output layer) to 10% (bottleneck) in Frobenius norm; the
network test therefore bounds the output difference by 2% of max |f(x)|, the
loss by 1%, and each layer's gradient by 15% in norm with a cosine
similarity of at least 0.99.  A wrong mask, operand or skip path moves these
by O(1).
"""
import math

import numpy as np
import pytest

import oracle.denoiser as dn
from tests.gpu_util import dev, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    import paper_2407_20692_amd.denoiser as m
    return m


def bf16_tensor(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(dev())


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else \
        t.cpu().numpy().astype(np.float64)


def rand_bf16(rng, shape, scale=1.0):
    return dn.round_bf16(rng.standard_normal(shape) * scale)


CONV_CASES = [
    # b, h, w, cin, cout, ks -- small grids: register-fed kernel
    (2, 9, 13, 8, 32, 3),
    (1, 16, 16, 32, 64, 3),
    (2, 7, 11, 96, 32, 3),
    (1, 12, 10, 32, 32, 1),
    (1, 4, 4, 384, 128, 3),
    # 1x1 layers whose weight gradients span several K tiles
    (2, 9, 13, 128, 64, 1),
    (1, 12, 10, 160, 32, 1),
    # LDS-staged 3x3 kernel: the first tile shape (rows x channels) whose
    # grid holds >= 512 work-groups (then 256, 128); every shape covered (8 x 128, 8 x 64,
    # 4 x 64, 16 x 32, 8 x 32, 4 x 32), ragged edges
    (16, 64, 64, 32, 128, 3),   # 8 x 128
    (8, 64, 64, 32, 128, 3),    # 8 x 64
    (9, 60, 62, 64, 64, 3),     # 4 x 64
    (16, 128, 64, 32, 32, 3),   # 16 x 32
    (8, 60, 62, 64, 64, 3),     # 8 x 32
    (16, 64, 64, 32, 32, 3),    # 8 x 32
    (16, 16, 16, 128, 256, 3),  # 4 x 32
    (8, 64, 60, 96, 32, 3),     # 4 x 32
    (16, 32, 32, 32, 32, 3),    # 4 x 32 at the 256-group threshold
    # all-taps 3x3 weight gradient: 64-column blocks with ragged rows and
    # columns, for 32 and 64 output channels
    (2, 21, 70, 32, 32, 3),
    (3, 9, 67, 64, 64, 3),
]


@pytest.mark.parametrize("case", CONV_CASES, ids=[str(c) for c in CONV_CASES])
def test_conv_forward_and_input_grad(nn, case):
    import torch
    b, h, w, cin, cout, ks = case
    log(f"conv {case}")
    rng = np.random.default_rng(hash(case) % 2**32)
    x = rand_bf16(rng, (b, h, w, cin))
    wt = rng.standard_normal((cout, ks, ks, cin)) / math.sqrt(cin * ks * ks)
    bias = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    mask = dn.round_bf16(rng.standard_normal((b, h, w, cout)))
    wq = dn.round_bf16(wt.astype(np.float32))
    wf, wtp = nn.pack_weights(torch.from_numpy(wt.astype(np.float32)).to(dev()))
    # forward, ReLU, mask
    out = nn.conv2d(bf16_tensor(x), wf, ks, cout, bias=torch.from_numpy(bias.astype(np.float32))
                    .to(dev()), mask=bf16_tensor(mask), relu=True)
    ref = dn.conv2d(x, wq, bias)
    S = dn.conv2d(np.abs(x), np.abs(wq), np.abs(bias))
    K = ks * ks * cin
    ref_out = np.where(mask > 0, np.maximum(ref, 0.0), 0.0)
    err = np.abs(host(out) - ref_out)
    bound = 2.0 ** -8 * np.abs(ref_out) + K * 2.0 ** -23 * S
    assert np.all(err <= bound), float((err - bound).max())
    # FP32 output, no activation
    of = torch.empty(b, h, w, cout, dtype=torch.float32, device=dev())
    nn.conv2d(bf16_tensor(x), wf, ks, cout, out_f32=of)
    ref0 = dn.conv2d(x, wq)
    S0 = dn.conv2d(np.abs(x), np.abs(wq))
    assert np.all(np.abs(host(of) - ref0) <= K * 2.0 ** -23 * S0 + 2.0 ** -24 * np.abs(ref0))
    # gradient with respect to the input: the same kernel on the flipped,
    # transposed weights (roles of cin and cout exchanged)
    if cin % 32 == 0:
        dy = rand_bf16(rng, (b, h, w, cout))
        dx = nn.conv2d(bf16_tensor(dy), wtp, ks, cin)
        refd = dn.conv2d_grad_input(dy, wq)
        Sd = dn.conv2d_grad_input(np.abs(dy), np.abs(wq))
        Kd = ks * ks * cout
        errd = np.abs(host(dx) - refd)
        assert np.all(errd <= 2.0 ** -8 * np.abs(refd) + Kd * 2.0 ** -23 * Sd)


@pytest.mark.parametrize("case", CONV_CASES, ids=[str(c) for c in CONV_CASES])
def test_conv_weight_and_bias_grad(nn, case):
    import torch
    b, h, w, cin, cout, ks = case
    log(f"wgrad {case}")
    rng = np.random.default_rng(7 + hash(case) % 2**31)
    x = rand_bf16(rng, (b, h, w, cin))
    dy = rand_bf16(rng, (b, h, w, cout))
    dw0 = rng.standard_normal((cout, ks, ks, cin)).astype(np.float32)
    dw = torch.from_numpy(dw0.copy()).to(dev())
    db0 = rng.standard_normal(cout).astype(np.float32)
    dbf = torch.from_numpy(db0.copy()).to(dev())
    ref = dw0 + dn.conv2d_grad_weight(x, dy, ks)
    S = np.abs(dw0) + dn.conv2d_grad_weight(np.abs(x), np.abs(dy), ks)
    M = b * h * w
    Sb = np.abs(dy).sum(axis=(0, 1, 2))
    xt, dyt = bf16_tensor(x), bf16_tensor(dy)
    # pixel splits added with FP32 atomics (no workspace)
    nn.conv2d_wgrad(xt, dyt, ks, dw, db=dbf)
    assert np.all(np.abs(host(dw) - ref) <= (M + 2) * 2.0 ** -23 * S)
    assert np.all(np.abs(host(dbf) - db0 - dn.bias_grad(dy)) <= (M + 2) * 2.0 ** -23 * (Sb + np.abs(db0)))
    # partial sums in a workspace, added in split order: same bound, and two
    # calls agree bit for bit
    ws = torch.empty(nn.conv2d_wgrad_workspace_size(b, h, w, cin, cout, ks), dtype=torch.uint8,
                     device=dev())
    runs = []
    for _ in range(2):
        dw2 = torch.from_numpy(dw0.copy()).to(dev())
        db2 = torch.from_numpy(db0.copy()).to(dev())
        nn.conv2d_wgrad(xt, dyt, ks, dw2, db=db2, workspace=ws)
        runs.append((host(dw2), host(db2)))
    assert np.all(np.abs(runs[0][0] - ref) <= (M + 2) * 2.0 ** -23 * S)
    assert np.all(np.abs(runs[0][1] - db0 - dn.bias_grad(dy)) <= (M + 2) * 2.0 ** -23 * (Sb + np.abs(db0)))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    # without a bias gradient the bias slots are neither written nor read
    dw3 = torch.from_numpy(dw0.copy()).to(dev())
    nn.conv2d_wgrad(xt, dyt, ks, dw3, workspace=ws)
    assert np.array_equal(host(dw3), runs[0][0])
    db = torch.zeros(cout, dtype=torch.float32, device=dev())
    nn.bias_grad(bf16_tensor(dy), db)
    assert np.all(np.abs(host(db) - dn.bias_grad(dy)) <= (M + 2) * 2.0 ** -23 * Sb)


def test_wgrad_workspace_too_small(nn):
    import torch
    from paper_2407_20692_amd.binding import CpiError
    b, h, w, cin, cout = 2, 16, 16, 32, 64
    need = nn.conv2d_wgrad_workspace_size(b, h, w, cin, cout, 3)
    assert need > 0
    x = torch.zeros(b, h, w, cin, dtype=torch.bfloat16, device=dev())
    dy = torch.zeros(b, h, w, cout, dtype=torch.bfloat16, device=dev())
    dw = torch.zeros(cout, 3, 3, cin, dtype=torch.float32, device=dev())
    ws = torch.empty(need - 4, dtype=torch.uint8, device=dev())
    with pytest.raises(CpiError) as e:
        nn.conv2d_wgrad(x, dy, 3, dw, workspace=ws)
    assert "workspace" in str(e.value)


def test_routing_kernels_bit_exact(nn):
    rng = np.random.default_rng(21)
    x = rand_bf16(rng, (2, 6, 10, 32))
    x[0, 0, 0, :] = x[0, 0, 1, :]                      # ties inside a window
    assert np.array_equal(host(nn.maxpool2(bf16_tensor(x))), dn.maxpool2(x))
    g = rand_bf16(rng, (2, 3, 5, 32))
    assert np.array_equal(host(nn.maxpool2_grad(bf16_tensor(x), bf16_tensor(g))),
                          dn.maxpool2_grad(x, g))
    u = rand_bf16(rng, (2, 3, 5, 64))
    assert np.array_equal(host(nn.upsample2(bf16_tensor(u))), dn.upsample2(u))
    a = rand_bf16(rng, (2, 3, 5, 64))
    c = rand_bf16(rng, (2, 3, 5, 32))
    cat = nn.concat(bf16_tensor(a), bf16_tensor(c))
    assert np.array_equal(host(cat), np.concatenate([a, c], axis=3))
    da, dc = nn.split(cat, 64)
    assert np.array_equal(host(da), a) and np.array_equal(host(dc), c)
    # fused upsampling + concatenation
    skip = rand_bf16(rng, (2, 6, 10, 32))
    uc = nn.upsample2_concat(bf16_tensor(u), bf16_tensor(skip))
    assert np.array_equal(host(uc), np.concatenate([dn.upsample2(u), skip], axis=3))


def test_upsample_grad_and_add_mask(nn):
    rng = np.random.default_rng(22)
    g = rand_bf16(rng, (2, 8, 6, 32))
    mask = rand_bf16(rng, (2, 4, 3, 32))
    ref = dn.round_bf16(dn.upsample2_grad(g)) * (mask > 0)
    got = host(nn.upsample2_grad(bf16_tensor(g), mask=bf16_tensor(mask)))
    S = dn.upsample2_grad(np.abs(g))
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 4 * 2.0 ** -23 * S)
    # fused gradient of upsampling + concatenation
    d = rand_bf16(rng, (2, 8, 6, 96))
    m2 = rand_bf16(rng, (2, 4, 3, 64))
    dlow, dskip = nn.upsample2_concat_grad(bf16_tensor(d), 64, mask=bf16_tensor(m2))
    assert np.array_equal(host(dskip), d[..., 64:])
    ref2 = dn.round_bf16(dn.upsample2_grad(d[..., :64])) * (m2 > 0)
    S2 = dn.upsample2_grad(np.abs(d[..., :64]))
    assert np.all(np.abs(host(dlow) - ref2) <= 2.0 ** -8 * np.abs(ref2) + 4 * 2.0 ** -23 * S2)
    a = rand_bf16(rng, (3, 5, 32))
    b = rand_bf16(rng, (3, 5, 32))
    m = rand_bf16(rng, (3, 5, 32))
    x = bf16_tensor(a)
    nn.add_mask(x, bf16_tensor(b), bf16_tensor(m))
    ref = (a + b) * (m > 0)
    assert np.all(np.abs(host(x) - ref) <= 2.0 ** -8 * np.abs(ref) + 2.0 ** -23 * (np.abs(a) + np.abs(b)))


def test_mse_and_adam(nn):
    import torch
    rng = np.random.default_rng(23)
    P, C = 1000, 32
    y = rng.standard_normal((P, C)).astype(np.float32)
    res = rng.standard_normal(P).astype(np.float32)
    t = rng.standard_normal(P).astype(np.float32)
    loss, dy = nn.mse(torch.from_numpy(y).to(dev()), torch.from_numpy(t).to(dev()),
                      residual=torch.from_numpy(res).to(dev()))
    z = y[:, 0].astype(np.float64) + res
    assert math.isclose(float(host(loss)), dn.mse(z, t), rel_tol=1e-5)
    gref = np.zeros((P, C))
    gref[:, 0] = dn.mse_grad(z, t)
    assert np.all(np.abs(host(dy) - gref) <= 2.0 ** -8 * np.abs(gref) + 1e-6 * np.abs(gref).max())
    n = 5000
    w = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    wd, md, vd = (torch.from_numpy(a.copy()).to(dev()) for a in (w, m, v))
    wr, mr, vr = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        nn.adam(wd, torch.from_numpy(g).to(dev()), md, vd, step, lr=1e-2)
        wr, mr, vr = dn.adam_step(wr, g.astype(np.float64), mr, vr, step, lr=1e-2)
    assert np.all(np.abs(host(wd) - wr) <= 1e-6 * np.abs(wr) + 1e-5 * 1e-2)


def _logical_params(nn, params_dev):
    """GPU parameter array -> oracle parameters {name: (w, b)} at logical sizes."""
    p = host(params_dev)
    out = {}
    for L in nn.layers():
        w = p[L.weight_offset:L.weight_offset + L.weight_count].reshape(L.cout, L.ks, L.ks, L.cin)
        b = p[L.bias_offset:L.bias_offset + L.cout]
        out[L.name] = (w[:L.cout_used, :, :, :L.cin_used].copy(), b[:L.cout_used].copy())
    return out


def _grad_logical(nn, g_dev):
    g = host(g_dev)
    out = {}
    for L in nn.layers():
        w = g[L.weight_offset:L.weight_offset + L.weight_count].reshape(L.cout, L.ks, L.ks, L.cin)
        b = g[L.bias_offset:L.bias_offset + L.cout]
        out[L.name] = (w, b)
    return out


def test_layer_table_matches_oracle(nn):
    infos = nn.layers()
    ref = dn.layers()
    assert [L.name for L in infos] == [L.name for L in ref]
    for L, R in zip(infos, ref):
        assert (L.cin_used, L.cout_used, L.ks) == (R.cin, R.cout, R.ks)
        assert L.cin % 8 == 0 and L.cout % 32 == 0
    # padded channels stay zero after init
    import torch
    p = nn.init_params(3, dev())
    for L in infos:
        w, b = nn.layer_view(p, L)
        assert torch.count_nonzero(w[L.cout_used:]) == 0
        assert torch.count_nonzero(w[..., L.cin_used:]) == 0


def _synthetic_planes(rng, b, h, w):
    yy, xx = np.mgrid[0:h, 0:w]
    t = np.stack([np.sin(xx / (2 + k)) * np.cos(yy / (3 + k)) + 0.3 * k for k in range(b)])
    return (t + 0.4 * rng.standard_normal(t.shape)).astype(np.float32), t.astype(np.float32)


# (8, 32, 32) and (4, 64, 64): the decoder's first convolutions read their
# concatenated input directly at levels 0 and 1 (grids large enough for the
# LDS-staged kernel) and through a written-out concatenation at level 2
@pytest.mark.parametrize("shape", [(2, 16, 16), (1, 24, 40), (8, 32, 32), (4, 64, 64)])
def test_network_forward_and_gradients(nn, shape):
    import torch
    b, h, w = shape
    log(f"network {shape}")
    rng = np.random.default_rng(31)
    net = nn.Denoiser(seed=5, device=dev())
    # non-zero biases so that every bias path is exercised
    for L in nn.layers():
        _, bb = nn.layer_view(net.params, L)
        bb[:L.cout_used] = torch.from_numpy(rng.standard_normal(L.cout_used).astype(np.float32)
                                            * 0.05).to(dev())
    params = _logical_params(nn, net.params)
    planes, targets = _synthetic_planes(rng, b, h, w)
    out = host(net.forward(torch.from_numpy(planes).to(dev())))
    ref = dn.denoise(params, planes)
    x, mu, sd = dn.normalize_planes(planes)
    f_ref = (ref - mu[:, None, None]) / sd[:, None, None] - x
    f_gpu = (out - mu[:, None, None]) / sd[:, None, None] - x
    err = np.abs(f_gpu - f_ref).max()
    log(f"  forward: max|f| {np.abs(f_ref).max():.4f}, max err {err:.3e}")
    assert err <= 2e-2 * np.abs(f_ref).max()
    loss, grads = net.gradients(torch.from_numpy(planes).to(dev()),
                                torch.from_numpy(targets).to(dev()))
    loss_ref, g_ref, _ = dn.loss_and_grads(params, planes, targets)
    assert math.isclose(float(host(loss)), loss_ref, rel_tol=1e-2)
    g = _grad_logical(nn, grads)
    for L in nn.layers():
        gw, gb = g[L.name]
        rw, rb = g_ref[L.name]
        # padded channels receive no gradient
        assert np.all(gw[L.cout_used:] == 0) and np.all(gw[..., L.cin_used:] == 0)
        gw = gw[:L.cout_used, :, :, :L.cin_used]
        ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
        eb = np.linalg.norm(gb[:L.cout_used] - rb) / max(np.linalg.norm(rb), 1e-30)
        cos = float(np.sum(gw * rw) / (np.linalg.norm(gw) * np.linalg.norm(rw)))
        log(f"  {L.name}: rel grad err w {ew:.2e} b {eb:.2e} cos {cos:.5f}")
        assert ew <= 0.15 and eb <= 0.15 and cos >= 0.99, L.name


def test_training_reduces_loss(nn):
    import torch
    rng = np.random.default_rng(41)
    net = nn.Denoiser(seed=1, device=dev())
    planes, targets = _synthetic_planes(rng, 8, 32, 32)
    p, t = torch.from_numpy(planes).to(dev()), torch.from_numpy(targets).to(dev())
    first = float(net.train_step(p, t, lr=1e-3))
    for _ in range(150):
        loss = net.train_step(p, t, lr=1e-3)
    last = float(loss)
    log(f"training: loss {first:.4f} -> {last:.4f}")
    assert np.isfinite(last) and last < 0.3 * first
    # the padded channels are still zero
    for L in nn.layers():
        w, _ = nn.layer_view(net.params, L)
        assert torch.count_nonzero(w[L.cout_used:]) == 0
        assert torch.count_nonzero(w[..., L.cin_used:]) == 0


def test_image_quality_matches_oracle(nn):
    import torch
    rng = np.random.default_rng(51)
    t = rng.random((3, 24, 30)).astype(np.float32)
    p = (t + 0.1 * rng.standard_normal(t.shape)).astype(np.float32)
    p[2] = t[2]
    psnr, ssim = nn.image_quality(torch.from_numpy(p).to(dev()), torch.from_numpy(t).to(dev()))
    psnr, ssim = host(psnr), host(ssim)
    for k in range(3):
        rp = dn.psnr(p[k], t[k])
        rs = dn.ssim(p[k], t[k])
        if math.isinf(rp):
            assert math.isinf(psnr[k])
        else:
            assert math.isclose(psnr[k], rp, rel_tol=1e-10)
        assert math.isclose(ssim[k], rs, rel_tol=1e-9, abs_tol=1e-12)
