"""The learned-bounds network's device kernels (bf16 MFMA forward, backward, AdamW) against
the FP64 reference with the same bfloat16 roundings.

Tolerances: the device accumulates in FP32 in MFMA order and the reference in FP64, so an
intermediate that sits within one FP32 rounding of a bfloat16 tie can round the other
way; each such flip moves one activation by one bf16 step (2^-8 relative).  Outputs of
order one therefore agree to about 1e-3 and are held to 1e-2; gradients, sums of many
such products, are held to 2e-2 in relative norm per parameter block.  The AdamW update
is elementwise FP32 arithmetic, held to 1e-5 relative; its bfloat16 repacking is exact."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from paper_2510_02639_amd import icrs

pytestmark = pytest.mark.gpu

NPF = icrs.MLP_PARAM_FLOATS


def _blob(p):
    """Padded FP32 blob of the header's layout from a reference parameter dict."""
    b = np.zeros(NPF, np.float32)
    W1 = np.zeros((128, 32))
    W1[:, :10] = p["W1"]
    W4 = np.zeros((16, 128))
    W4[:4] = p["W4"]
    b4 = np.zeros(16)
    b4[:4] = p["b4"]
    parts = [W1, p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], W4, b4]
    o = 0
    for a in parts:
        a = np.asarray(a).ravel()
        b[o:o + a.size] = a
        o += a.size
    assert o == NPF
    return b


def _unblob(b):
    b = np.asarray(b, np.float64)
    W1 = b[0:4096].reshape(128, 32)
    o = 4096
    out = {"W1": W1[:, :10]}
    pad = {"W1": W1[:, 10:]}
    for name, n in (("b1", 128), ("W2", 16384), ("b2", 128), ("W3", 16384), ("b3", 128)):
        out[name] = b[o:o + n].reshape(128, 128) if name.startswith("W") else b[o:o + n]
        o += n
    W4 = b[o:o + 2048].reshape(16, 128)
    out["W4"], pad["W4"] = W4[:4], W4[4:]
    o += 2048
    out["b4"], pad["b4"] = b[o:o + 4], b[o + 4:o + 16]
    return out, pad


def _setup(seed, m):
    rng = np.random.default_rng(seed)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in M.init_params(seed).items()}
    x = rng.normal(size=(m, 10)) * rng.uniform(0.5, 3, size=10) + rng.uniform(-2, 2, size=10)
    t = rng.normal(size=(m, 4)) * 0.7 + 0.3
    norm = np.zeros(32, np.float32)
    norm[0:10] = rng.uniform(-2, 2, size=10)
    norm[10:20] = rng.uniform(0.5, 3, size=10)
    norm[20:24] = [0.3, -0.1, 0.2, 0.0]
    norm[24:28] = [0.7, 1.3, 0.9, 1.1]
    x = x.astype(np.float32)
    t = t.astype(np.float32)
    x_std = (x.astype(np.float64) - norm[0:10]) / norm[10:20]
    t_std = (t.astype(np.float64) - norm[20:24]) / norm[24:28]
    h = icrs.Handle()
    dev = {k: torch.tensor(v, device="cuda") for k, v in (("params", _blob(p)), ("norm", norm), ("x", x), ("t", t))}
    dev["packed"] = torch.empty(icrs.MLP_PACKED_HALFS, dtype=torch.int16, device="cuda")
    h.mlp_pack(dev["params"], dev["packed"])
    return h, p, x_std, t_std, norm, dev


@pytest.mark.parametrize("m", [1, 64, 200, 4099])
def test_forward_matches_reference(m):
    h, p, x_std, _, norm, dev = _setup(11 + m, m)
    y = h.mlp_forward(dev["packed"], dev["params"], dev["norm"], dev["x"]).cpu().numpy().astype(np.float64)
    y_std = (y - norm[20:24]) / norm[24:28]
    yq, _ = M.forward(p, x_std, quantize=True)
    y64, _ = M.forward(p, x_std, quantize=False)
    err = np.abs(y_std - yq).max()
    print(f"m={m}: max |y - ref_bf16| = {err:.2e}, max |y - ref_fp64| = {np.abs(y_std - y64).max():.2e}", flush=True)
    assert err <= 1e-2
    assert np.abs(y_std - y64).max() <= 5e-2 * max(1.0, np.abs(y64).max())


def test_packed_weights_are_bf16_of_master():
    h, p, _, _, _, dev = _setup(3, 64)
    pk = dev["packed"].cpu().numpy().view(np.uint16)
    blob = _blob(p)
    bits = M.bf16(blob).astype(np.float32).view(np.uint32) >> 16
    W1 = bits[0:4096]
    assert np.array_equal(pk[0:4096], W1)
    W2 = bits[4224:4224 + 16384].reshape(128, 128)
    assert np.array_equal(pk[4096:4096 + 16384].reshape(128, 128), W2)
    # transposed copy of W2 follows W1, W2, W3, W4
    o = 4096 + 16384 + 16384 + 2048
    assert np.array_equal(pk[o:o + 16384].reshape(128, 128), W2.T)


@pytest.mark.parametrize("m", [64, 333, 5000])
def test_loss_and_gradient_match_reference(m):
    h, p, x_std, t_std, _, dev = _setup(21 + m, m)
    grad, loss = h.mlp_loss_grad(dev["packed"], dev["params"], dev["norm"], dev["x"], dev["t"])
    g_dev, pad = _unblob(grad.cpu().numpy())
    lq, gq = M.loss_and_grad(p, x_std, t_std, quantize=True)
    assert abs(loss.item() - lq) <= 1e-3 * lq
    for k in gq:
        rel = np.linalg.norm(g_dev[k] - gq[k]) / np.linalg.norm(gq[k])
        print(f"m={m} {k}: rel err {rel:.2e}", flush=True)
        assert rel <= 2e-2, k
    for k, v in pad.items():
        assert np.all(v == 0), k
    # deterministic: a second call gives the same bits
    grad2, loss2 = h.mlp_loss_grad(dev["packed"], dev["params"], dev["norm"], dev["x"], dev["t"])
    assert torch.equal(grad, grad2) and torch.equal(loss, loss2)


def test_adamw_matches_reference():
    h, p, x_std, t_std, _, dev = _setup(5, 256)
    m_dev = torch.zeros(NPF, dtype=torch.float32, device="cuda")
    v_dev = torch.zeros_like(m_dev)
    pr, mr, vr = p, {k: np.zeros_like(v) for k, v in p.items()}, {k: np.zeros_like(v) for k, v in p.items()}
    for step in (1, 2, 3):
        grad, _ = h.mlp_loss_grad(dev["packed"], dev["params"], dev["norm"], dev["x"], dev["t"])
        g, _ = _unblob(grad.cpu().numpy())
        h.mlp_adamw(dev["params"], grad, m_dev, v_dev, step, 1e-3, weight_decay=0.01, packed=dev["packed"])
        pr, mr, vr = M.adamw_step(pr, g, mr, vr, step, 1e-3, weight_decay=0.01)
        got, pad = _unblob(dev["params"].cpu().numpy())
        for k in pr:
            assert np.allclose(got[k], pr[k], rtol=1e-5, atol=1e-7), (step, k)
        for k, v in pad.items():
            assert np.all(v == 0)
        pr = {k: v.astype(np.float32).astype(np.float64) for k, v in got.items()}
    pk = dev["packed"].cpu().numpy().view(np.uint16)
    bits = M.bf16(dev["params"].cpu().numpy()).astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(pk[0:4096], bits[0:4096])


def test_training_on_device_fits_a_smooth_map():
    """A few hundred AdamW steps of the device kernels fit a smooth 10 -> 4 map."""
    rng = np.random.default_rng(7)
    m = 4096
    x = rng.normal(size=(m, 10)).astype(np.float32)
    A = rng.normal(size=(10, 4)) / 3
    t = (np.tanh(x @ A) + 0.1 * np.sin(x[:, :4] * 2)).astype(np.float32)
    norm = np.zeros(32, np.float32)
    norm[10:20] = 1.0
    norm[24:28] = 1.0
    h = icrs.Handle()
    params = torch.tensor(_blob(M.init_params(8)), device="cuda")
    packed = torch.empty(icrs.MLP_PACKED_HALFS, dtype=torch.int16, device="cuda")
    h.mlp_pack(params, packed)
    nd, xd, td = (torch.tensor(a, device="cuda") for a in (norm, x, t))
    mm, vv = torch.zeros_like(params), torch.zeros_like(params)
    losses = []
    for step in range(1, 301):
        grad, loss = h.mlp_loss_grad(packed, params, nd, xd, td)
        losses.append(loss.item())
        h.mlp_adamw(params, grad, mm, vv, step, 3e-3, packed=packed)
    print(f"loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.05 * losses[0]


def test_argument_errors():
    h = icrs.Handle()
    x = torch.zeros((0, 10), dtype=torch.float32, device="cuda")
    y = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    assert icrs.lib().icrs_mlp_forward(h._h, None, None, None, 0, None, None) == 0
    assert icrs.lib().icrs_mlp_loss_grad(h._h, None, None, None, 0, None, None, None, None, None, 0) == -1
    assert icrs.lib().icrs_mlp_adamw(h._h, None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 0.0, None) == -1
    del x, y
