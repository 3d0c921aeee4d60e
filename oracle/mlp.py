"""MLP reference for the learned con2prim guess (test infrastructure only).

Network 5 -> 64 -> 64 -> 1 with ReLU, evaluated in float64 with the same
rounding points as the GPU path (round to nearest even to bfloat16):
standardised inputs, weights w1/w2/w3, and both hidden activations after the
ReLU; biases and the output stay unrounded.  `bf16=False` switches every
rounding off, which turns the network into a smooth function of its
parameters (used to pin the hand-written backward pass by finite
differences).

Parameter vector order: W1[64][5], b1[64], W2[64][64], b2[64], w3[64], b3.
Normalisation vector: x_mean[5], x_std[5], y_mean, y_std (inputs are
standardised as (x - x_mean) * binary32(1 / x_std)).
Features of a conserved state (D, S, tau), E = tau + D, s = |S|:
    [log(D/E), s/E, log(1 - s/E), log(tau/E), log((tau (tau + 2D) - s^2) / E^2)]
(the last is log((E^2 - D^2 - s^2)/E^2), a direct measure of the internal energy);
target: (log(p/E) - y_mean) / y_std.
"""
from __future__ import annotations

import numpy as np

IN, HID = 5, 64
NPARAM = HID * IN + HID + HID * HID + HID + HID + 1


def bf16_rne(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32 values.
    Definition: keep the top 16 bits of the binary32 pattern after adding
    0x7FFF plus the lowest kept bit; NaN stays NaN."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), np.float32(np.nan), out)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + HID * IN].reshape(HID, IN); o += HID * IN
    b1 = p[o:o + HID]; o += HID
    W2 = p[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = p[o:o + HID]; o += HID
    w3 = p[o:o + HID]; o += HID
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]])


def features(cons) -> np.ndarray:
    """raw features [n, 5] (float64) of conserved states cons [5, n]"""
    D, Sx, Sy, Sz, tau = np.asarray(cons, dtype=np.float64)
    E = tau + D
    s2 = Sx * Sx + Sy * Sy + Sz * Sz
    sE = np.sqrt(s2) / E
    return np.stack([np.log(D / E), sE, np.log(1.0 - sE), np.log(tau / E),
                     np.log((tau * (tau + 2.0 * D) - s2) / (E * E))], axis=1)


def standardise(x, norm, bf16=True):
    """(x - mean) * (1/std) in binary32 (x first rounded to binary32; the
    reciprocal is the correctly rounded binary32 quotient 1/std), then bf16.
    The product by the reciprocal is within 1.5 ulp of the quotient and is
    what the network defines as its input."""
    n32 = np.asarray(norm, dtype=np.float32)
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    inv = np.float32(1.0) / n32[5:10]
    z = (x32 - n32[:5]) * inv
    return bf16_rne(z).astype(np.float64) if bf16 else z.astype(np.float64)


def forward(params, norm, x, bf16=True, keep=False):
    """yhat for raw features x [n, 5]; keep=True also returns activations"""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    if bf16:
        W1, W2, w3 = (bf16_rne(np.float32(w)).astype(np.float64) for w in (W1, W2, w3))
        xb = standardise(x, norm, True)
    else:
        n = np.asarray(norm, dtype=np.float64)
        xb = (np.asarray(x, dtype=np.float64) - n[:5]) / n[5:10]
    a1 = xb @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    if bf16:
        h1 = bf16_rne(h1.astype(np.float32)).astype(np.float64)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    if bf16:
        h2 = bf16_rne(h2.astype(np.float32)).astype(np.float64)
    y = h2 @ w3 + b3
    if keep:
        return y, (xb, h1, h2, W1, W2, w3)
    return y


def loss_and_grad(params, norm, x, t, bf16=True):
    """mean squared error of the standardised target and its gradient
    (backward written by hand; rounding treated as the identity, ReLU
    derivative 1 where the activation is positive)"""
    y, (xb, h1, h2, W1, W2, w3) = forward(params, norm, x, bf16, keep=True)
    n = len(y)
    d = y - np.asarray(t, dtype=np.float64)
    loss = np.mean(d * d)
    dy = 2.0 * d / n
    gw3 = h2.T @ dy
    gb3 = np.sum(dy)
    dh2 = (dy[:, None] * w3[None, :]) * (h2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (h1 > 0)
    gW1 = dh1.T @ xb
    gb1 = dh1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(params, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def guess(params, norm, cons, bf16=True):
    """learned pressure guess E exp(y_mean + y_std yhat) for cons [5, n]"""
    x = features(cons)
    y = forward(params, norm, x, bf16)
    if bf16:
        y = y.astype(np.float32).astype(np.float64)  # the GPU output is binary32
    E = cons[4] + cons[0]
    return E * np.exp(float(np.float32(norm[10])) + float(np.float32(norm[11])) * y)


def target(cons, p) -> np.ndarray:
    """training target log(p / E), E = tau + D, in float64, rounded to float32"""
    cons = np.asarray(cons, dtype=np.float64)
    E = cons[4] + cons[0]
    return np.log(np.asarray(p, dtype=np.float64) / E).astype(np.float32)


def fit_norm(x, y) -> np.ndarray:
    """normalisation block of a training set: per feature column and for the
    target, the mean and the standard deviation with divisor n - 1 (feature
    deviations floored at 1e-6), in float64, rounded to float32:
    [x_mean(5), x_std(5), y_mean, y_std]"""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xm = x.mean(axis=0)
    xs = np.maximum(x.std(axis=0, ddof=1), 1e-6)
    return np.concatenate([xm, xs, [y.mean(), y.std(ddof=1)]]).astype(np.float32)


def standardise_target(y, norm) -> np.ndarray:
    """(y - y_mean) / y_std in float64 with the float32 statistics, rounded to
    float32"""
    n = np.asarray(norm, dtype=np.float32).astype(np.float64)
    return ((np.asarray(y, dtype=np.float32).astype(np.float64) - n[10]) / n[11]).astype(np.float32)
