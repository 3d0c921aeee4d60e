"""Training of the learned con2prim guess with the library's own kernels.

Pairs (conserved state, pressure) come from the seeded SRHD primitive
distribution of the SRHD workload (rho, eps log-uniform in [1e-3, 10],
Lorentz factor uniform in [1, 10], isotropic velocity) mapped to conserved
variables by the input generator.  Everything after that runs in the library
(torch only allocates the device buffers):
  pb_mlp_prepare             raw features and the target log(p/E),
  pb_mlp_fit_norm            their means and standard deviations,
  pb_mlp_standardise_target  the standardised target,
  pb_mlp_train_epoch         per epoch, Adam steps on batches of a seeded
                             permutation of the rows (forward, backward and
                             update on the matrix cores), cosine learning rate.
"""
from __future__ import annotations

import math

import numpy as np

from . import MLP_HID, MLP_IN, MLP_NPARAM, Mlp, pb_mlp_prepare
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
    """raw features x [n, 5] and targets log(p/E) [n] (float32, device, made by
    the library), conserved states [5, n] (float64, device)"""
    import torch
    cons, p = I.srhd_training_pairs(seed, n)
    c = torch.from_numpy(np.ascontiguousarray(cons)).to(device)
    pt = torch.from_numpy(np.ascontiguousarray(p)).to(device)
    x, y = pb_mlp_prepare(c, pt)
    return x, y, c


# placeholder statistics until pb_mlp_fit_norm replaces them on the device
_UNIT_NORM = np.array([0.0] * 5 + [1.0] * 5 + [0.0, 1.0], np.float32)


def train(n_pairs=1 << 22, epochs=20, batch=8192, lr=3e-3, seed=2024, data_seed=77, device="cuda", log=None):
    """Returns (Mlp, history dict): per-epoch mean batch loss, step count and
    the fitted normalisation.  Cosine learning-rate decay over all steps."""
    import torch
    x, y, _ = dataset(data_seed, n_pairs, device)
    net = Mlp(he_init(seed), _UNIT_NORM)
    net.fit_norm(x, y)
    t = net.standardise_target(y)
    steps_per_epoch = n_pairs // batch
    total = epochs * steps_per_epoch
    loss_sum = torch.zeros(epochs, dtype=torch.float64, device=device)
    for ep in range(epochs):
        net.train_epoch(x, t, batch, seed, ep, lr, ep * steps_per_epoch, total, loss_sum=loss_sum[ep:])
        if log:
            log(f"epoch {ep + 1}/{epochs} queued")
    sums = loss_sum.cpu().numpy()
    hist = {"epoch_loss": [float(v) / steps_per_epoch for v in sums], "steps": total,
            "norm": net.get_params()[1]}
    return net, hist
