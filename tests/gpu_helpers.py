"""Shared helpers of the GPU parity tests (they compare the HIP library,
called through its C ABI, with the CPU oracle on the same seeded inputs)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(batch, g, o):
    """per unknown v: max over cells |g - o| / max over cells |o| (the
    relative error metric every tolerance below refers to)."""
    N = batch.n_unknowns
    off = batch.offsets()
    C = batch.cells()
    errs = np.zeros(N)
    scale = np.zeros(N)
    for k in range(batch.K):
        a = g[off[k] * N:(off[k] + C[k]) * N].reshape(N, -1)
        b = o[off[k] * N:(off[k] + C[k]) * N].reshape(N, -1)
        errs = np.maximum(errs, np.max(np.abs(a - b), axis=1))
        scale = np.maximum(scale, np.max(np.abs(b), axis=1))
    return errs / np.where(scale > 0, scale, 1.0)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
