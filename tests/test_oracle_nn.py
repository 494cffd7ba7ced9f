"""Pins for the denoiser oracle: convolution against torch's float64 conv2d
(a library routine), gradients against central finite differences, the loss
and Adam against their definitions on hand values."""
import numpy as np
import pytest
import torch

from oracle import nn


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64))


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_library_conv2d(stride):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 10, 12, 5))
    W = rng.normal(size=(7, 3, 3, 5))
    b = rng.normal(size=7)
    got = nn.conv_fwd(x, W, b, stride)
    ref = torch.nn.functional.conv2d(_t(x).permute(0, 3, 1, 2), _t(W).permute(0, 3, 1, 2),
                                     _t(b), stride=stride, padding=1).permute(0, 2, 3, 1)
    np.testing.assert_allclose(got, ref.numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_gradients_match_library_autograd(stride):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 10, 4))
    W = rng.normal(size=(6, 3, 3, 4))
    b = rng.normal(size=6)
    xt = _t(x).permute(0, 3, 1, 2).requires_grad_(True)
    Wt = _t(W).permute(0, 3, 1, 2).requires_grad_(True)
    bt = _t(b).requires_grad_(True)
    y = torch.nn.functional.conv2d(xt, Wt, bt, stride=stride, padding=1)
    dy = rng.normal(size=y.shape)
    y.backward(_t(dy))
    dy_nhwc = dy.transpose(0, 2, 3, 1)
    dW, db = nn.conv_wgrad(x, dy_nhwc, stride)
    dx = nn.conv_dgrad(dy_nhwc, W, x.shape, stride)
    np.testing.assert_allclose(dW, Wt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-10, atol=1e-10)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0], np.float32)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6)
    assert list(nn.bf16(vals)) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0]
    # against torch's bfloat16 conversion
    rng = np.random.default_rng(3)
    r = rng.normal(size=10000).astype(np.float32) * 10
    ref = torch.from_numpy(r).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16(r), ref)


def _exact_net(params, x, target):
    """The same network without BF16 rounding, for finite differences."""
    W, b = nn.unpack(params)
    c1 = np.maximum(nn.conv_fwd(x, W["c1"], b["c1"]), 0)
    c2 = np.maximum(nn.conv_fwd(c1, W["c2"], b["c2"], 2), 0)
    c3 = np.maximum(nn.conv_fwd(c2, W["c3"], b["c3"]), 0)
    c4 = np.maximum(nn.conv_fwd(nn.up2(c3), W["c4"], b["c4"]), 0)
    c5 = np.maximum(nn.conv_fwd(np.concatenate([c1, c4], -1), W["c5"], b["c5"]), 0)
    out = x[..., :3] + nn.conv_fwd(c5, W["c6"], b["c6"])
    return nn.loss(out, target)


def test_network_gradient_central_differences(monkeypatch):
    # with BF16 rounding switched off the oracle's backward is the exact
    # gradient of the float64 network: check it by central differences
    monkeypatch.setattr(nn, "bf16", lambda a: np.asarray(a, np.float64))
    rng = np.random.default_rng(4)
    params = nn.init_params(5).astype(np.float64)
    params[nn.param_layout()[0]["c6"][0]:] *= 10    # non-trivial last layer
    x = rng.uniform(0, 1, size=(1, 6, 8, 8))
    x[..., 5:] = 0
    t = rng.uniform(0, 1, size=(1, 6, 8, 3))
    L, g = nn.backward(params, x, t)
    assert L == pytest.approx(_exact_net(params, x, t), rel=1e-12)
    idx = rng.choice(len(params), 60, replace=False)
    h = 1e-6
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        fd = (_exact_net(p1, x, t) - _exact_net(p2, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_loss_and_grad_definition():
    out = np.array([[0.5, 1.0, 0.0]])
    t = np.array([[0.4, 1.0, 0.1]])
    want = np.mean([(0.1 ** 2) / (0.16 + 0.01), 0.0, 0.01 / (0.01 + 0.01)])
    assert nn.loss(out, t) == pytest.approx(want, rel=1e-14)
    g = nn.loss_grad(out, t)
    assert g[0, 0] == pytest.approx(2 * 0.1 / 0.17 / 3, rel=1e-12)


def test_adam_first_step_is_signed_lr():
    # after one bias-corrected step the update is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    new, m, v = nn.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(new, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # and it matches torch.optim.Adam on a second step
    pt = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, eps=1e-8)
    for step, gg in enumerate([g, g * 0.5 + 0.1], start=1):
        pt.grad = torch.tensor(gg)
        opt.step()
    p2, m2, v2 = nn.adam_step(new, g * 0.5 + 0.1, m, v, 2, 0.01)
    np.testing.assert_allclose(p2, pt.detach().numpy(), rtol=1e-12)


def _torch_bf16(t):
    return t.to(torch.bfloat16).to(torch.float64)


def test_bf16_gradient_option_matches_autograd_with_rounding_hooks():
    # the option that rounds every inter-layer gradient to BF16, against
    # torch's autograd of the same float64 network: activations rounded to
    # BF16 in the forward pass with an identity gradient, and a hook rounding
    # the gradient of each convolution's output (pre-activation) to BF16
    rng = np.random.default_rng(6)
    params = nn.init_params(7).astype(np.float64)
    params[nn.param_layout()[0]["c6"][0]:] *= 10
    x = nn.bf16(rng.uniform(0, 1, size=(2, 8, 12, 8)))
    x[..., 5:] = 0
    t = rng.uniform(0, 1, size=(2, 8, 12, 3))
    L, g = nn.backward(params, x, t, bf16_grads=True)
    W, b = nn.unpack(params)
    Wt = {k: _torch_bf16(_t(v).permute(0, 3, 1, 2)).requires_grad_(True) for k, v in W.items()}
    bt = {k: _t(v).requires_grad_(True) for k, v in b.items()}

    def conv(a, name, stride=1, relu=True):
        y = torch.nn.functional.conv2d(a, Wt[name], bt[name], stride=stride, padding=1)
        y.register_hook(_torch_bf16)
        if not relu:
            return y
        r = torch.relu(y)
        return r + (_torch_bf16(r) - r).detach()     # rounded value, identity gradient

    xt = _t(x).permute(0, 3, 1, 2)
    c1 = conv(xt, "c1")
    c2 = conv(c1, "c2", 2)
    c3 = conv(c2, "c3")
    c4 = conv(torch.repeat_interleave(torch.repeat_interleave(c3, 2, 2), 2, 3), "c4")
    c5 = conv(torch.cat([c1, c4], 1), "c5")
    out = xt[:, :3] + conv(c5, "c6", relu=False)
    tt = _t(t).permute(0, 3, 1, 2)
    Lt = torch.mean((out - tt) ** 2 / (tt * tt + 0.01))
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    lay, _ = nn.param_layout()
    for name, (ow, ob, cin, cout) in lay.items():
        gw = Wt[name].grad.permute(0, 2, 3, 1).numpy().ravel()
        np.testing.assert_allclose(g[ow:ob], gw, rtol=1e-9, atol=1e-12 * np.abs(gw).max())
        np.testing.assert_allclose(g[ob:ob + cout], bt[name].grad.numpy(), rtol=1e-9,
                                   atol=1e-12 * np.abs(gw).max())
    # and the rounding moves the gradient by no more than BF16 precision allows
    _, g_exact = nn.backward(params, x, t)
    assert np.linalg.norm(g - g_exact) <= 2e-2 * np.linalg.norm(g_exact)
    assert not np.array_equal(g, g_exact)
