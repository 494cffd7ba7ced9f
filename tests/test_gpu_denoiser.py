"""GPU parity of the denoiser's BF16-MFMA kernels against the oracle: each
convolution (forward, data and weight gradient) on the same BF16 inputs, the
whole training step's loss and gradient, and the Adam update."""
import numpy as np
import pytest
import torch

import synth
from oracle import nn
from paper_2504_04564_amd import _build, denoiser, vdbc
from synth import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return vdbc.load()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _bf(rng, shape, scale=1.0, relu=False):
    x = rng.normal(size=shape).astype(np.float32) * scale
    if relu:
        x = np.maximum(x, 0)
    t = torch.from_numpy(x).to(torch.bfloat16)
    return t.cuda(), t.to(torch.float64).numpy()


CONV_CASES = [  # (ca, cb, up, stride, cout, n, hs, ws)
    (8, 0, 0, 1, 32, 2, 18, 22),
    (32, 0, 0, 2, 64, 1, 20, 34),
    (64, 0, 0, 1, 64, 2, 9, 13),
    (64, 0, 1, 1, 32, 1, 7, 11),
    (32, 32, 0, 1, 32, 2, 14, 10),
    (32, 0, 0, 1, 3, 1, 17, 19),
    (32, 0, 0, 1, 40, 1, 12, 15),   # 33..48 output channels take the four-tile kernel
    (16, 8, 0, 1, 20, 1, 9, 70),    # 24 input channels in a 32-channel block, three 32-column tiles
    (40, 8, 1, 1, 16, 1, 5, 9),     # 48 input channels in two 32-channel blocks, upsampled
    (16, 8, 1, 2, 24, 2, 7, 9),     # stride 2 through an upsampled concat, odd sizes
]


@pytest.mark.parametrize("ca,cb,up,stride,cout,n,hs,ws", CONV_CASES)
def test_conv_forward(ca, cb, up, stride, cout, n, hs, ws):
    rng = np.random.default_rng(ca + 3 * cout + hs)
    a, a64 = _bf(rng, (n, hs, ws, ca))
    b, b64 = _bf(rng, (n, hs, ws, cb)) if cb else (None, None)
    w, w64 = _bf(rng, (cout, 3, 3, ca + cb), 0.2)
    bias = torch.from_numpy(rng.normal(size=cout).astype(np.float32)).cuda()
    x64 = a64 if not cb else np.concatenate([a64, b64], -1)
    if up:
        x64 = nn.up2(x64)
    ref = nn.conv_fwd(x64, w64, bias.cpu().numpy().astype(np.float64), stride)
    got = vdbc.conv3x3(a, b, up, stride, w, bias, cout, relu=False, out_f32=True)
    assert rel(got.cpu().numpy(), ref) <= 1e-5
    got_bf = vdbc.conv3x3(a, b, up, stride, w, bias, cout, relu=True)
    assert rel(got_bf.float().cpu().numpy(), np.maximum(ref, 0)) <= 1e-2


@pytest.mark.parametrize("ca,cb,up,stride,cout,n,hs,ws", CONV_CASES)
def test_conv_gradients(ca, cb, up, stride, cout, n, hs, ws):
    rng = np.random.default_rng(7 * ca + cout + ws)
    cin = ca + cb
    a, a64 = _bf(rng, (n, hs, ws, ca))
    b, b64 = _bf(rng, (n, hs, ws, cb)) if cb else (None, None)
    w, w64 = _bf(rng, (cout, 3, 3, cin), 0.2)
    hv, wv = (2 * hs, 2 * ws) if up else (hs, ws)
    ho, wo = (hv - 1) // stride + 1, (wv - 1) // stride + 1
    coutp = (cout + 7) // 8 * 8
    dz_np = rng.normal(size=(n, ho, wo, coutp)).astype(np.float32)
    dz_np[..., cout:] = 0
    dz = torch.from_numpy(dz_np).to(torch.bfloat16)
    dz64 = dz.to(torch.float64).numpy()[..., :cout]
    dz = dz.cuda()
    x64 = a64 if not cb else np.concatenate([a64, b64], -1)
    if up:
        x64 = nn.up2(x64)
    dx = vdbc.conv3x3_dgrad(dz, cout, w, cin, stride, hv, wv).cpu().numpy()
    assert rel(dx, nn.conv_dgrad(dz64, w64, x64.shape, stride)) <= 1e-5
    dw, db = vdbc.conv3x3_wgrad(a, b, up, stride, dz, cout)
    rdw, rdb = nn.conv_wgrad(x64, dz64, stride)
    assert rel(dw.cpu().numpy(), rdw) <= 1e-5
    assert rel(db.cpu().numpy(), rdb) <= 1e-5


# Sizes at which a weight-gradient chunk spans many rows of its band: 64
# input channels over 257 x 511 pixels (two channel blocks, ragged last
# band and column tile), the first layer's 8 input channels at batch
# 8 x 512^2, and the stride-2 layer at batch 8 from 256 x 255 (odd width).
WGRAD_LARGE = [(64, 0, 0, 1, 64, 1, 257, 511), (8, 0, 0, 1, 32, 8, 512, 512), (32, 0, 0, 2, 64, 8, 256, 255)]


@pytest.mark.parametrize("ca,cb,up,stride,cout,n,hs,ws", WGRAD_LARGE)
def test_conv_weight_gradient_large(ca, cb, up, stride, cout, n, hs, ws):
    rng = np.random.default_rng(ca + cout + hs)
    a, a64 = _bf(rng, (n, hs, ws, ca))
    ho, wo = (hs - 1) // stride + 1, (ws - 1) // stride + 1
    dz_np = rng.normal(size=(n, ho, wo, cout)).astype(np.float32)
    dz = torch.from_numpy(dz_np).to(torch.bfloat16)
    dz64 = dz.to(torch.float64).numpy()
    dw, db = vdbc.conv3x3_wgrad(a, None, up, stride, dz.cuda(), cout)
    rdw, rdb = nn.conv_wgrad(a64, dz64, stride)
    assert rel(dw.cpu().numpy(), rdw) <= 1e-5
    assert rel(db.cpu().numpy(), rdb) <= 1e-5


def _batch(rng, n, h, w):
    x = np.zeros((n, h, w, 8), np.float32)
    x[..., :3] = rng.uniform(0, 1.2, size=(n, h, w, 3))
    x[..., 3] = rng.uniform(0, 1, size=(n, h, w))
    x[..., 4] = rng.integers(0, 2, size=(n, h, w))
    t = np.clip(x[..., :3] + rng.normal(scale=0.1, size=(n, h, w, 3)), 0, None).astype(np.float32)
    return x, t


def test_train_step_loss_and_gradient_vs_oracle():
    rng = np.random.default_rng(11)
    n, h, w = 2, 24, 32
    x, t = _batch(rng, n, h, w)
    params = nn.init_params(3)
    params[nn.param_layout()[0]["c6"][0]:] *= 10
    dn = vdbc.Denoiser(params)
    xb = torch.from_numpy(x).to(torch.bfloat16).cuda()
    tt = torch.from_numpy(t).cuda()
    grad = torch.empty(len(params), dtype=torch.float32, device="cuda")
    loss = dn.train_step(xb, tt, lr=0.0, grad_out=grad).item()
    L, g = nn.backward(params.astype(np.float64), xb.cpu().to(torch.float64).numpy(), t)
    assert abs(loss - L) <= 1e-3 * L
    gg = grad.cpu().numpy()
    lay, _ = nn.param_layout()
    for name, (ow, ob, cin, cout) in lay.items():
        assert rel(gg[ow:ob], g[ow:ob]) <= 2e-2, name
        assert rel(gg[ob:ob + cout], g[ob:ob + cout]) <= 2e-2, name
    assert rel(gg, g) <= 1e-2
    # the GPU stores each inter-layer gradient in BF16: against the oracle
    # that rounds at the same points the gradients agree far more closely
    # (what is left is FP32 accumulation and the rare BF16 rounding decision
    # that it flips)
    Lq, gq = nn.backward(params.astype(np.float64), xb.cpu().to(torch.float64).numpy(), t,
                         bf16_grads=True)
    worst = {}
    for name, (ow, ob, cin, cout) in lay.items():
        worst[name] = max(rel(gg[ow:ob], gq[ow:ob]), rel(gg[ob:ob + cout], gq[ob:ob + cout]))
    print("per-layer relative gradient error vs the BF16-gradient oracle:", worst)
    assert max(worst.values()) <= 2e-3, worst
    assert rel(gg, gq) <= 1e-3
    # inference output equals the oracle forward
    out = dn(xb).cpu().numpy()
    ref, _ = nn.forward(params.astype(np.float64), xb.cpu().to(torch.float64).numpy())
    assert rel(out, ref) <= 1e-2


def test_adam_update_matches_oracle_formula():
    rng = np.random.default_rng(12)
    n, h, w = 1, 16, 16
    x, t = _batch(rng, n, h, w)
    params = nn.init_params(4)
    dn = vdbc.Denoiser(params)
    xb = torch.from_numpy(x).to(torch.bfloat16).cuda()
    tt = torch.from_numpy(t).cuda()
    p = params.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    grad = torch.empty(len(params), dtype=torch.float32, device="cuda")
    for step in (1, 2, 3):
        before = dn.params.cpu().numpy().astype(np.float64)
        dn.train_step(xb, tt, lr=1e-3, grad_out=grad)
        g = grad.cpu().numpy().astype(np.float64)
        p, m, v = nn.adam_step(before, g, m, v, step, 1e-3)
        after = dn.params.cpu().numpy()
        assert np.max(np.abs(after - p)) <= 1e-6 + 1e-5 * np.max(np.abs(p))
        assert torch.equal(dn.wbf16, dn.params.to(torch.bfloat16))


def test_training_reduces_loss():
    rng = np.random.default_rng(13)
    n, h, w = 4, 32, 32
    x, t = _batch(rng, n, h, w)
    dn = vdbc.Denoiser(seed=5)
    xb = torch.from_numpy(x).to(torch.bfloat16).cuda()
    tt = torch.from_numpy(t).cuda()
    first = dn.train_step(xb, tt, lr=2e-3).item()
    for _ in range(60):
        last = dn.train_step(xb, tt, lr=2e-3).item()
    assert np.isfinite(last) and last < 0.7 * first


def test_pack_layout():
    rgba = torch.rand((2, 6, 4, 4), device="cuda")
    aov = torch.rand((2, 6, 4, 2), device="cuda")
    x = vdbc.denoise_pack(rgba, aov)
    want = torch.cat([rgba[..., :3], aov, torch.zeros((2, 6, 4, 3), device="cuda")], -1)
    assert torch.equal(x, want.to(torch.bfloat16))


def test_render_pair_input_and_target():
    # one training example: the network input packs the spp_in render and its
    # AOVs, the target is an independent spp_ref render (other seed)
    v = synth.cloud_volume((48, 48, 48), seed=1001)
    g = vdbc.Grid(vdbc.encode(v, 0.10)[0])
    cam = scenes.orbit_camera(g.dims, 40, 24)
    med = scenes.pt_medium(64.0)
    x, ref = denoiser.render_pair(g, cam, med, 4, 32, seed=77)
    assert x.shape == (24, 40, 8) and x.dtype == torch.bfloat16
    assert ref.shape == (24, 40, 3) and ref.dtype == torch.float32
    prm = dict(max_bounces=8, macrocell=16)
    lo, aov = vdbc.render(g, cam, med, dict(prm, spp=4, seed=77), vdbc.MODE_PT, aov=True)
    assert torch.equal(x[..., :3], lo[..., :3].to(torch.bfloat16))
    assert torch.equal(x[..., 3:5], aov.to(torch.bfloat16))
    assert torch.all(x[..., 5:] == 0)
    hi = vdbc.render(g, cam, med, dict(prm, spp=32, seed=77 ^ 0x9E3779B97F4A7C15), vdbc.MODE_PT)
    assert torch.equal(ref, hi[..., :3])
    same_seed = vdbc.render(g, cam, med, dict(prm, spp=32, seed=77), vdbc.MODE_PT)
    assert not torch.equal(ref, same_seed[..., :3])


def test_trained_denoiser_beats_the_plain_render():
    # the learned part against the method without it: trained on GPU-rendered
    # pairs (96 crops of 256^2 from 16 seeded clouds at 1:10, 4-spp inputs,
    # 512-spp targets, 1500 Adam steps of batch 8), then evaluated on a
    # held-out cloud against a 1024-spp reference: the denoised 4-spp image
    # has a lower relMSE than the plain 4-spp and the plain 64-spp renders,
    # in less time than the 64-spp render
    rng = np.random.default_rng(1000)
    med = scenes.pt_medium(64.0)
    xs, ts = [], []
    for i in range(16):
        side = int(rng.integers(128, 257))
        g = vdbc.Grid(vdbc.encode(synth.cloud_volume((side, side, side), seed=1000 + i), 0.10)[0])
        for k in range(6):
            cam = scenes.orbit_camera(g.dims, 256, 256, azimuth_deg=float(rng.uniform(0, 360)),
                                      elevation_deg=float(rng.uniform(-30, 45)),
                                      distance=float(rng.uniform(1.2, 2.0)))
            x, t = denoiser.render_pair(g, cam, med, 4, 512, seed=7919 * i + k)
            xs.append(x)
            ts.append(t)
    X, T = torch.stack(xs), torch.stack(ts)
    dn = vdbc.Denoiser(seed=5)
    losses = denoiser.train(dn, X, T, steps=1500, batch=8, lr=1e-3, seed=1)
    assert np.all(np.isfinite(losses)) and np.mean(losses[-50:]) < 0.5 * np.mean(losses[:50])
    v = synth.cloud_volume((256, 256, 256), seed=5000)
    g = vdbc.Grid(vdbc.encode(v, 0.10)[0])
    cam = scenes.orbit_camera(g.dims, 256, 256, azimuth_deg=40.0)
    e = denoiser.evaluate(dn, g, cam, med, seed=31)
    assert e["relmse_denoised"] < e["relmse_plain_lo"]
    assert e["relmse_denoised"] <= e["relmse_plain_hi"], e
    assert e["ms_denoised_pipeline"] < e["ms_plain_hi"], e


def test_conv_outputs_at_unaligned_addresses():
    # outputs that are not 16-byte (FP32) or 8-byte (BF16) aligned take the
    # staged epilogues' element-by-element stores; results as at aligned ones
    import ctypes as C
    L = vdbc._nn()
    rng = np.random.default_rng(91)
    n, h, w, cin, cout = 1, 12, 40, 32, 32
    a, a64 = _bf(rng, (n, h, w, cin))
    wt, w64 = _bf(rng, (cout, 3, 3, cin), 0.2)
    bias = torch.from_numpy(rng.normal(size=cout).astype(np.float32)).cuda()
    want = vdbc.conv3x3(a, None, 0, 1, wt, bias, cout, relu=True)
    raw = torch.zeros(n * h * w * cout + 8, dtype=torch.bfloat16, device="cuda")
    ptr = raw.data_ptr() + 2   # 2-byte aligned only
    assert L.vdbc_conv3x3(a.data_ptr(), cin, None, 0, 0, n, h, w, 1, wt.data_ptr(), bias.data_ptr(), cout, 1,
                          C.c_void_p(ptr), None, vdbc._stream()) == 0
    torch.cuda.synchronize()
    got = raw[1:1 + n * h * w * cout].view(n, h, w, cout)
    assert torch.equal(got.view(torch.int16), want.view(torch.int16))
    # data gradient into an FP32 buffer offset by one float
    dz_np = rng.normal(size=(n, h, w, cout)).astype(np.float32)
    dz = torch.from_numpy(dz_np).to(torch.bfloat16).cuda()
    ref = vdbc.conv3x3_dgrad(dz, cout, wt, cin, 1, h, w)
    ws = C.c_uint64(0)
    assert L.vdbc_conv3x3_grad_workspace(cin, cout, n, h, w, C.byref(ws)) == 0
    buf, wptr = vdbc._aligned_empty(int(ws.value), dz.device)
    dxr = torch.zeros(n * h * w * cin + 4, dtype=torch.float32, device="cuda")
    assert L.vdbc_conv3x3_dgrad(dz.data_ptr(), cout, cout, n, h, w, wt.data_ptr(), cin, 1, h, w,
                                C.c_void_p(dxr.data_ptr() + 4), wptr, int(ws.value), vdbc._stream()) == 0
    torch.cuda.synchronize()
    got_dx = dxr[1:1 + n * h * w * cin].view(n, h, w, cin)
    assert torch.equal(got_dx, ref)
