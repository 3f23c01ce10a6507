"""Pins of the FP64 learned-bounds network reference against library routines (PyTorch's
float64 Linear/GELU/autograd/AdamW, its bfloat16 cast) and finite differences."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle import mlp_ref as M


def _data(m=37, seed=1):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(m, M.N_IN)), rng.normal(size=(m, M.N_OUT))


def test_param_count():
    assert M.N_PARAMS == 34948


def test_gelu_matches_torch_tanh_form_and_its_derivative():
    x = np.linspace(-9, 9, 2001)
    ref = F.gelu(torch.tensor(x), approximate="tanh").numpy()
    assert np.max(np.abs(M.gelu(x) - ref)) < 1e-15 * 10
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(M.gelu_grad(x) - fd)) < 1e-8
    assert M.gelu(0.0) == 0.0 and abs(M.gelu(30.0) - 30.0) < 1e-12 and abs(M.gelu(-30.0)) < 1e-12


def test_bf16_rounding_matches_torch_cast():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, size=5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -7.5e-39]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)
    assert np.array_equal(M.bf16(M.bf16(x)), M.bf16(x))


def _torch_net(p):
    return {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}


def _torch_forward(tp, x):
    h = torch.tensor(x)
    for l in (1, 2, 3):
        h = F.gelu(F.linear(h, tp[f"W{l}"], tp[f"b{l}"]), approximate="tanh")
    return F.linear(h, tp["W4"], tp["b4"])


def test_forward_and_gradients_match_torch_float64():
    p = M.init_params(3)
    x, t = _data()
    y, _ = M.forward(p, x)
    tp = _torch_net(p)
    yt = _torch_forward(tp, x)
    assert np.max(np.abs(y - yt.detach().numpy())) < 1e-13
    loss, g = M.loss_and_grad(p, x, t)
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-14
    for k in tp:
        assert np.max(np.abs(g[k] - tp[k].grad.numpy())) < 1e-14, k


def test_gradients_match_central_differences():
    p = M.init_params(4)
    x, t = _data(11, 5)
    _, g = M.loss_and_grad(p, x, t)
    rng = np.random.default_rng(6)
    for name, shape in M.SHAPES:
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in shape)
            h = 1e-6
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (M.loss_and_grad(pp, x, t)[0] - M.loss_and_grad(pm, x, t)[0]) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd)), (name, idx)


def test_quantized_network_stays_within_bf16_error():
    p = M.init_params(7)
    x, t = _data(64, 8)
    y, _ = M.forward(p, x)
    yq, _ = M.forward(p, x, quantize=True)
    assert np.max(np.abs(yq - y)) <= 2e-2 * np.max(np.abs(y))
    _, g = M.loss_and_grad(p, x, t)
    _, gq = M.loss_and_grad(p, x, t, quantize=True)
    for k in g:
        assert np.linalg.norm(gq[k] - g[k]) <= 3e-2 * np.linalg.norm(g[k]), k


def test_adamw_matches_torch_optimizer():
    p = M.init_params(9)
    x, t = _data(16, 10)
    tp = _torch_net(p)
    opt = torch.optim.AdamW([{"params": [tp[k] for k in tp if k.startswith("W")], "weight_decay": 0.05},
                             {"params": [tp[k] for k in tp if k.startswith("b")], "weight_decay": 0.0}],
                            lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    for step in range(1, 4):
        _, g = M.loss_and_grad(p, x, t)
        p, m, v = M.adamw_step(p, g, m, v, step, 1e-2, weight_decay=0.05)
        opt.zero_grad()
        torch.mean((_torch_forward(tp, x) - torch.tensor(t)) ** 2).backward()
        opt.step()
        for k in p:
            assert np.max(np.abs(p[k] - tp[k].detach().numpy())) < 1e-12, (step, k)
