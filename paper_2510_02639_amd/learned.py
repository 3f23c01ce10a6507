"""Learned grid bounds: data from the plain path, device training, the model the learned
path reads.  Not part of the paper's method (it extends its sector step).

Every computation runs in the HIP library (``icrs_image_bounds`` for the data,
``icrs_mlp_loss_grad`` / ``icrs_mlp_adamw`` for training, ``icrs_mlp_forward`` for
calibration); this module sequences the calls and keeps the tensors.

Training data are the plain path's own per-image extents (the limb images of the sector
step, given to the nearest centre image) on epochs drawn like the planetary batch but
from their own seed, restricted to epochs where the image count does not change across
the source (the only epochs the learned path serves).  Targets are ln(offset / sigma),
sigma = rho / |1 - |kappa|| the image's linearised size; inputs and targets are
standardised with the training set's mean and deviation.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np
import torch

from . import icrs, workloads

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "bounds_mlp.npz")


def init_blob(seed: int) -> np.ndarray:
    """Padded FP32 parameter blob (layout of include/icrs.h) with each layer drawn
    uniform in +-1/sqrt(fan_in) (weights and biases)."""
    rng = np.random.default_rng(seed)
    b = np.zeros(icrs.MLP_PARAM_FLOATS, np.float32)
    o = 0

    def put(shape, pad_shape, fan_in):
        nonlocal o
        a = np.zeros(pad_shape, np.float32)
        bound = 1.0 / np.sqrt(fan_in)
        sl = tuple(slice(0, s) for s in shape)
        a[sl] = rng.uniform(-bound, bound, size=shape)
        b[o:o + a.size] = a.ravel()
        o += a.size

    put((128, 10), (128, 32), 10)
    put((128,), (128,), 10)
    for _ in range(2):
        put((128, 128), (128, 128), 128)
        put((128,), (128,), 128)
    put((4, 128), (16, 128), 128)
    put((4,), (16,), 128)
    assert o == icrs.MLP_PARAM_FLOATS
    return b


@dataclasses.dataclass
class BoundsModel:
    params: torch.Tensor      # FP32 master blob (CUDA)
    norm: torch.Tensor        # [32] FP32 (CUDA)
    log_safety: float
    packed: torch.Tensor = None

    def __post_init__(self):
        if self.packed is None:
            self.packed = torch.empty(icrs.MLP_PACKED_HALFS, dtype=torch.int16, device=self.params.device)
            self.repack()

    def repack(self, handle=None):
        (handle or icrs.Handle()).mlp_pack(self.params, self.packed)

    def save(self, path=DEFAULT_PATH):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(),
                 log_safety=np.array(self.log_safety))

    @staticmethod
    def load(path=DEFAULT_PATH, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            return BoundsModel(torch.tensor(z["params"], device=device), torch.tensor(z["norm"], device=device),
                               float(z["log_safety"]))


TARGET_MAX = 3.0   # rows with an extent beyond e^3 sigma are not linear-size images: not learned


def training_rows(handle, w: workloads.Workload):
    """(x [M, 10], y [M, 4]) CUDA float32: the valid image rows of a workload (epochs with a
    constant image count over the limb; images whose four targets stay <= TARGET_MAX)."""
    t = torch.tensor(w.t, device="cuda")
    feat, tgt, nimg, flags = handle.image_bounds(w.params, w.offsets, t)
    mi = feat.shape[1]
    j = torch.arange(mi, device="cuda").unsqueeze(0)
    mask = (flags == 0).unsqueeze(1) & (j < nimg.unsqueeze(1)) & (tgt <= TARGET_MAX).all(dim=2)
    return feat[mask].contiguous(), tgt[mask].contiguous()


def fit_norm(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    norm = torch.zeros(32, dtype=torch.float32, device=x.device)
    norm[0:10] = x.mean(0)
    norm[10:20] = x.std(0).clamp_min(1e-3)
    norm[20:24] = y.mean(0)
    norm[24:28] = y.std(0).clamp_min(1e-3)
    return norm


def train(handle, x, y, steps=6000, batch=16384, lr=2e-3, weight_decay=1e-4, seed=50, log_every=0):
    """AdamW on the device kernels; cosine decay of the step size.  Returns (model, losses)."""
    norm = fit_norm(x, y)
    model = BoundsModel(torch.tensor(init_blob(seed), device="cuda"), norm, 0.0)
    m = torch.zeros_like(model.params)
    v = torch.zeros_like(model.params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = x.shape[0]
    ws = torch.empty(icrs.lib().icrs_mlp_workspace_bytes(min(batch, n)), dtype=torch.uint8, device="cuda")
    grad = torch.empty_like(model.params)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    perm, pos = torch.randperm(n, generator=gen, device="cuda"), 0
    for step in range(1, steps + 1):
        if pos + batch > n:
            perm, pos = torch.randperm(n, generator=gen, device="cuda"), 0
        idx = perm[pos:pos + min(batch, n)]
        pos += idx.numel()
        xb, yb = x.index_select(0, idx), y.index_select(0, idx)
        handle.mlp_loss_grad(model.packed, model.params, model.norm, xb, yb, workspace=ws, grad=grad, loss=loss)
        a = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps))
        handle.mlp_adamw(model.params, grad, m, v, step, a, weight_decay=weight_decay, packed=model.packed)
        if log_every and (step % log_every == 0 or step == 1):
            losses.append((step, loss.item()))
    losses.append((steps, loss.item()))
    return model, losses


def calibrate(handle, model, x, y, coverage=0.99):
    """Set log_safety so that exp(prediction + log_safety) covers all four targets on a
    `coverage` fraction of rows.  Returns (log_safety, per-output RMS error)."""
    pred = handle.mlp_forward(model.packed, model.params, model.norm, x)
    gap = (y - pred).max(dim=1).values
    model.log_safety = float(torch.quantile(gap.double(), coverage).item())
    rms = ((y - pred) ** 2).mean(0).sqrt().cpu().numpy()
    return model.log_safety, rms


def train_default(n_events=8192, n_epochs=100, steps=6000, seed=50, verbose=False):
    """The shipped model: planetary-batch draws of seed 50 (rho log-uniform in
    [10^-3.5, 10^-2]), n_epochs per event clustered at the caustic crossings; 10% of the
    events held out for calibration."""
    w = workloads.binary_batch(seed, n_events, n_epochs_fixed=n_epochs, name="bounds-training")
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    n_val = n_events // 10
    x_tr, y_tr = training_rows(h, w.subset(range(n_val, n_events)))
    x_va, y_va = training_rows(h, w.subset(range(n_val)))
    if verbose:
        print(f"[learned] {x_tr.shape[0]} training rows, {x_va.shape[0]} validation rows", flush=True)
    model, losses = train(h, x_tr, y_tr, steps=steps, seed=seed, log_every=500 if verbose else 0)
    ls, rms = calibrate(h, model, x_va, y_va)
    if verbose:
        print(f"[learned] losses {losses}; log_safety {ls:.3f}; validation RMS {rms}", flush=True)
    return model, {"train_rows": int(x_tr.shape[0]), "val_rows": int(x_va.shape[0]), "losses": losses,
                   "log_safety": ls, "val_rms": rms.tolist()}
