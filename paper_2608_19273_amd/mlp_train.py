"""Training of the learned con2prim guess with the library's own kernels.

Pairs (conserved state, pressure) come from the seeded SRHD primitive
distribution of the SRHD workload (rho, eps log-uniform in [1e-3, 10],
Lorentz factor uniform in [1, 10], isotropic velocity) mapped to conserved
variables by the input generator.  Features are computed on the GPU by
pb_mlp_features; the target is log(p/E), standardised.  Each optimisation
step is one pb_mlp_train_step call (forward, backward, weight gradients and an
Adam update on the device).
"""
from __future__ import annotations

import math

import numpy as np

from . import MLP_HID, MLP_IN, MLP_NPARAM, Mlp, pb_mlp_features
from . import inputs as I


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, SplitMix64 +
    Box-Muller draws."""
    w1 = I.normal(I.substream(seed, 1), MLP_HID * MLP_IN) * math.sqrt(2.0 / MLP_IN)
    w2 = I.normal(I.substream(seed, 2), MLP_HID * MLP_HID) * math.sqrt(2.0 / MLP_HID)
    w3 = I.normal(I.substream(seed, 3), MLP_HID) * math.sqrt(1.0 / MLP_HID)
    p = np.concatenate([w1, np.zeros(MLP_HID), w2, np.zeros(MLP_HID), w3, [0.0]]).astype(np.float32)
    assert p.size == MLP_NPARAM
    return p


def dataset(seed: int, n: int, device="cuda"):
    """raw features x [n, 5] (float32, device), log(p/E) [n] (float64, device),
    conserved states [5, n] (float64, device)"""
    import torch
    cons, p = I.srhd_training_pairs(seed, n)
    c = torch.from_numpy(np.ascontiguousarray(cons)).to(device)
    x = pb_mlp_features(c)
    E = c[4] + c[0]
    y = torch.log(torch.from_numpy(p).to(device) / E)
    return x, y, c


def train(n_pairs=1 << 22, epochs=20, batch=8192, lr=3e-3, seed=2024, data_seed=77, device="cuda", log=None):
    """Returns (Mlp, history dict).  Cosine learning-rate decay over all steps."""
    import torch
    x, y, _ = dataset(data_seed, n_pairs, device)
    xm = x.double().mean(0)
    xs = x.double().std(0).clamp_min(1e-6)
    ym, ys = y.mean(), y.std()
    norm = np.concatenate([xm.cpu().numpy(), xs.cpu().numpy(), [ym.item(), ys.item()]]).astype(np.float32)
    t = ((y - float(norm[10])) / float(norm[11])).float()
    net = Mlp(he_init(seed), norm)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    steps_per_epoch = n_pairs // batch
    total = epochs * steps_per_epoch
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    hist = {"epoch_loss": []}
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n_pairs, generator=g, device=device)
        acc = torch.zeros((), dtype=torch.float64, device=device)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            step += 1
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * (step - 1) / total))
            net.train_step(xb, tb, lr_t, step, loss=loss)
            acc += loss[0].double()
        hist["epoch_loss"].append(acc.item() / steps_per_epoch)
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean batch loss {hist['epoch_loss'][-1]:.3e}")
    hist["steps"] = step
    hist["norm"] = norm
    return net, hist
