"""Oracle for the learned denoiser: 3x3 convolutions (forward, data and weight
gradients), the 6-layer U-Net, the relative-MSE loss and one Adam step, in
float64 from BF16-rounded operands.

TEST INFRASTRUCTURE ONLY (see oracle/oracle.h): the product's kernels never
import this module.

The denoiser is not part of the paper (which renders without one); the
network is this project's own extension and is fixed as follows.  Tensors are
NHWC.  Input x has 8 channels: RGB of a low-sample-count render, first-scatter
depth fraction, primary transmittance, three zeros.

    c1 = relu(conv(x,  W1, b1))                   H   x W   x 32
    c2 = relu(conv(c1, W2, b2, stride 2))         H/2 x W/2 x 64
    c3 = relu(conv(c2, W3, b3))                   H/2 x W/2 x 64
    c4 = relu(conv(up2(c3), W4, b4))              H   x W   x 32   (nearest x2)
    c5 = relu(conv(concat(c1, c4), W5, b5))       H   x W   x 32
    c6 = conv(c5, W6, b6)                         H   x W   x 3
    out = x[..., :3] + c6

Every conv is 3x3 with zero padding 1; weights are W[co][ky][kx][ci].
Activations are stored in BF16 (round to nearest even) between layers; each
layer accumulates in float64 here (the GPU accumulates in float32).
Loss = mean over pixels and RGB of (out - t)^2 / (t^2 + 0.01).
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # (name, cin, cout, stride, relu)
    ("c1", 8, 32, 1, True),
    ("c2", 32, 64, 2, True),
    ("c3", 64, 64, 1, True),
    ("c4", 64, 32, 1, True),
    ("c5", 64, 32, 1, True),
    ("c6", 32, 3, 1, False),
]


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def param_layout():
    """Offsets of each layer's weights and bias in the flat float32 vector:
    for every layer W (cout*9*cin) then b (cout)."""
    out, off = {}, 0
    for name, cin, cout, stride, relu in LAYERS:
        out[name] = (off, off + cout * 9 * cin, cin, cout)
        off += cout * 9 * cin + cout
    return out, off


def unpack(params: np.ndarray):
    lay, _ = param_layout()
    W, b = {}, {}
    for name, (ow, ob, cin, cout) in lay.items():
        W[name] = params[ow:ob].reshape(cout, 3, 3, cin).astype(np.float64)
        b[name] = params[ob:ob + cout].astype(np.float64)
    return W, b


def _patches(x: np.ndarray, stride: int) -> np.ndarray:
    """im2col: (N, Ho, Wo, 3, 3, C) neighbourhoods with zero padding 1."""
    n, h, w, c = x.shape
    p = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    out = np.empty((n, ho, wo, 3, 3, c), dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            out[:, :, :, ky, kx, :] = p[:, ky:ky + stride * (ho - 1) + 1:stride,
                                        kx:kx + stride * (wo - 1) + 1:stride, :]
    return out


def conv_fwd(x, W, b, stride=1):
    """y[n,oy,ox,co] = b[co] + sum W[co,ky,kx,ci] x[n, s*oy+ky-1, s*ox+kx-1, ci]."""
    P = _patches(np.asarray(x, np.float64), stride)
    n, ho, wo = P.shape[:3]
    cout = W.shape[0]
    y = P.reshape(n * ho * wo, -1) @ np.asarray(W, np.float64).reshape(cout, -1).T
    return y.reshape(n, ho, wo, cout) + np.asarray(b, np.float64)


def conv_wgrad(x, dy, stride=1):
    """dW[co,ky,kx,ci] = sum over output pixels dy * x(patch); db = sum dy."""
    P = _patches(np.asarray(x, np.float64), stride)
    n, ho, wo = P.shape[:3]
    cout = dy.shape[-1]
    g = np.asarray(dy, np.float64).reshape(-1, cout)
    dW = g.T @ P.reshape(n * ho * wo, -1)
    return dW.reshape(cout, 3, 3, x.shape[-1]), g.sum(axis=0)


def conv_dgrad(dy, W, in_shape, stride=1):
    """Gradient with respect to the input: scatter of dy through W."""
    n, h, w, cin = in_shape
    dy = np.asarray(dy, np.float64)
    Wf = np.asarray(W, np.float64)
    ho, wo = dy.shape[1], dy.shape[2]
    dxp = np.zeros((n, h + 2, w + 2, cin))
    for ky in range(3):
        for kx in range(3):
            contrib = dy @ Wf[:, ky, kx, :]          # (n, ho, wo, cin)
            dxp[:, ky:ky + stride * (ho - 1) + 1:stride,
                kx:kx + stride * (wo - 1) + 1:stride, :] += contrib
    return dxp[:, 1:h + 1, 1:w + 1, :]


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dx):
    n, h, w, c = dx.shape
    return dx.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def forward(params, x):
    """Returns (out, acts) where acts holds the BF16-rounded activations."""
    W, b = unpack(params)
    Wq = {k: bf16(v) for k, v in W.items()}
    a = {"x": bf16(x)}
    a["c1"] = bf16(np.maximum(conv_fwd(a["x"], Wq["c1"], b["c1"]), 0))
    a["c2"] = bf16(np.maximum(conv_fwd(a["c1"], Wq["c2"], b["c2"], 2), 0))
    a["c3"] = bf16(np.maximum(conv_fwd(a["c2"], Wq["c3"], b["c3"]), 0))
    a["u3"] = up2(a["c3"])
    a["c4"] = bf16(np.maximum(conv_fwd(a["u3"], Wq["c4"], b["c4"]), 0))
    a["cat"] = np.concatenate([a["c1"], a["c4"]], axis=-1)
    a["c5"] = bf16(np.maximum(conv_fwd(a["cat"], Wq["c5"], b["c5"]), 0))
    a["c6"] = conv_fwd(a["c5"], Wq["c6"], b["c6"])
    out = a["x"][..., :3] + a["c6"]
    return out, a


def loss(out, target):
    t = np.asarray(target, np.float64)
    return float(np.mean((out - t) ** 2 / (t * t + 0.01)))


def loss_grad(out, target):
    t = np.asarray(target, np.float64)
    return 2.0 * (out - t) / (t * t + 0.01) / out.size


def backward(params, x, target, bf16_grads: bool = False):
    """Loss and the gradient of every parameter (flat float64 vector) of the
    network whose forward pass uses the BF16-rounded weights and activations;
    the gradient itself is exact (float64, no rounding).  With bf16_grads the
    gradient with respect to each convolution's output (after the ReLU
    mask) is rounded to BF16 before it is propagated further, the precision
    in which a BF16 training step stores these tensors; everything else stays
    float64."""
    W, b = unpack(params)
    Wq = {k: bf16(v) for k, v in W.items()}
    out, a = forward(params, x)
    L = loss(out, target)
    q = bf16 if bf16_grads else (lambda v: v)
    g = {}
    d6 = q(loss_grad(out, target))
    g["c6"] = conv_wgrad(a["c5"], d6)
    d5 = q(conv_dgrad(d6, Wq["c6"], a["c5"].shape) * (a["c5"] > 0))
    g["c5"] = conv_wgrad(a["cat"], d5)
    dcat = conv_dgrad(d5, Wq["c5"], a["cat"].shape)
    d1 = dcat[..., :32]
    d4 = q(dcat[..., 32:] * (a["c4"] > 0))
    g["c4"] = conv_wgrad(a["u3"], d4)
    d3 = q(up2_backward(conv_dgrad(d4, Wq["c4"], a["u3"].shape)) * (a["c3"] > 0))
    g["c3"] = conv_wgrad(a["c2"], d3)
    d2 = q(conv_dgrad(d3, Wq["c3"], a["c2"].shape) * (a["c2"] > 0))
    g["c2"] = conv_wgrad(a["c1"], d2, 2)
    d1 = q((d1 + conv_dgrad(d2, Wq["c2"], a["c1"].shape, 2)) * (a["c1"] > 0))
    g["c1"] = conv_wgrad(a["x"], d1)
    lay, total = param_layout()
    grad = np.zeros(total)
    for name, (ow, ob, cin, cout) in lay.items():
        grad[ow:ob] = g[name][0].ravel()
        grad[ob:ob + cout] = g[name][1]
    return L, grad


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015), bias-corrected, step counted
    from 1; returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, zero weights
    for the three padding input channels of c1; float32."""
    lay, total = param_layout()
    rng = np.random.default_rng(seed)
    p = np.zeros(total, np.float32)
    for name, (ow, ob, cin, cout) in lay.items():
        fan_in = 9 * (5 if name == "c1" else cin)
        w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(cout, 3, 3, cin)).astype(np.float32)
        if name == "c1":
            w[..., 5:] = 0.0
        if name == "c6":
            w *= 0.1
        p[ow:ob] = w.ravel()
    return p
