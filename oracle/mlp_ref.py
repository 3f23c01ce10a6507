"""Plain FP64 reference of the learned-bounds network (numpy).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product path; it shares
no code with the HIP library.  The network is not in the paper: it is the small
multilayer perceptron that predicts a polar grid box for each point-source image, so the
limb images of the paper's sector step need not all be solved.

Network: 10 inputs -> 128 -> 128 -> 128 -> 4 outputs, GELU after each hidden layer (tanh
form of Hendrycks & Gimpel, 2016), 34 948 parameters.  Inputs are standardised with a
fixed mean/scale, outputs are standardised targets; the training loss is the mean squared
error over the rows and the four outputs.

``quantize=True`` applies, in FP64, the same bfloat16 roundings the device kernels take
(operands of every matrix product and the error signals between layers), so the device
result can be held to accumulation-order differences; ``quantize=False`` is the exact
FP64 network, pinned by finite differences.

Parameter layout (a flat dict here; the device's padded blob is rebuilt in the tests):
W1 [128, 10], b1 [128], W2 [128, 128], b2, W3 [128, 128], b3, W4 [4, 128], b4 [4].
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 10, 128, 4
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_OUT, N_HID)), ("b4", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 34 948
_C = np.sqrt(2.0 / np.pi)
_A = 0.044715


def gelu(x):
    """x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(_C * (x + _A * x ** 3)))


def gelu_grad(x):
    t = np.tanh(_C * (x + _A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _C * (1.0 + 3.0 * _A * x * x)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.  Values are
    first rounded to float32, as the device holds them there before narrowing."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def init_params(seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (PyTorch's Linear rule)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        fan_in = shape[1] if name.startswith("W") else (N_IN if name == "b1" else N_HID)
        b = 1.0 / np.sqrt(fan_in)
        p[name] = rng.uniform(-b, b, size=shape)
    return p


def _q(x, quantize):
    return bf16(x) if quantize else np.asarray(x, dtype=np.float64)


def forward(p, x_std, quantize=False):
    """Standardised inputs [M, 10] -> standardised outputs [M, 4], plus the cache the
    backward pass reads."""
    h0 = _q(x_std, quantize)
    cache = {"h0": h0}
    h = h0
    for l in (1, 2, 3):
        pre = h @ _q(p[f"W{l}"], quantize).T + p[f"b{l}"]
        h = _q(gelu(pre), quantize)
        cache[f"g{l}"] = _q(gelu_grad(pre), quantize)
        cache[f"h{l}"] = h
    y = h @ _q(p["W4"], quantize).T + p["b4"]
    return y, cache


def loss_and_grad(p, x_std, t_std, quantize=False):
    """L = mean over rows and outputs of (y - t)^2; returns (L, dict of dL/dparam)."""
    y, c = forward(p, x_std, quantize)
    m = x_std.shape[0]
    diff = y - t_std
    loss = float(np.sum(diff * diff) / (N_OUT * m))
    dy = _q(2.0 * diff / (N_OUT * m), quantize)
    g = {"W4": dy.T @ c["h3"], "b4": dy.sum(axis=0)}
    dp = dy
    w_next = "W4"
    for l in (3, 2, 1):
        dh = dp @ _q(p[w_next], quantize)
        dp = _q(dh * c[f"g{l}"], quantize)
        g[f"W{l}"] = dp.T @ c[f"h{l - 1}"]
        g[f"b{l}"] = dp.sum(axis=0)
        w_next = f"W{l}"
    return loss, g


def adamw_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW step (Loshchilov & Hutter): decoupled decay on the weight matrices only
    (biases are not decayed); bias-corrected moments.  Returns new (p, m, v) dicts."""
    p2, m2, v2 = {}, {}, {}
    for name, _ in SHAPES:
        m2[name] = beta1 * m[name] + (1.0 - beta1) * g[name]
        v2[name] = beta2 * v[name] + (1.0 - beta2) * g[name] ** 2
        mh = m2[name] / (1.0 - beta1 ** step)
        vh = v2[name] / (1.0 - beta2 ** step)
        decay = weight_decay if name.startswith("W") else 0.0
        p2[name] = p[name] - lr * decay * p[name] - lr * mh / (np.sqrt(vh) + eps)
    return p2, m2, v2
