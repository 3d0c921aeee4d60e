"""Pins of the MLP reference: bfloat16 rounding against torch's own
conversion, a network with a closed-form output, and the hand-written
backward pass against central finite differences."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2608_19273_amd import inputs as I


def test_bf16_rne_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    x = np.concatenate([I.normal(3, 20000).astype(np.float32) * 100,
                        np.float32([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 65504.0, 1e-30, 0.0])])
    ours = M.bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(ours, ref)
    assert M.bf16_rne(np.float32(1.0 + 2 ** -8)) == 1.0          # tie to even (down)
    assert M.bf16_rne(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6  # tie to even (up)


def test_closed_form_abs_network():
    """Hidden unit 0 = x0, unit 1 = -x0 (after the ReLU: |x0| split), layer 2
    copies them, w3 = (1, 1): the output is |x0| exactly (values that bf16
    holds exactly)."""
    W1 = np.zeros((64, 5)); W1[0, 0] = 1.0; W1[1, 0] = -1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    w3 = np.zeros(64); w3[0] = 1.0; w3[1] = 1.0
    p = M.pack(W1, np.zeros(64), W2, np.zeros(64), w3, 0.25)
    norm = np.array([0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 1], np.float32)
    x = np.zeros((6, 5)); x[:, 0] = [-3.0, -0.5, 0.0, 0.75, 2.0, 1.5]
    for bf in (True, False):
        np.testing.assert_array_equal(M.forward(p, norm, x, bf16=bf), np.abs(x[:, 0]) + 0.25)


def test_backward_against_finite_differences():
    rng_p = I.normal(5, M.NPARAM) * 0.3
    norm = np.array([0.1, -0.2, 0.3, 0.0, 0.5, 1.1, 0.9, 1.3, 0.7, 1.0, -2.0, 3.0])
    x = I.normal(6, 40 * 5).reshape(40, 5)
    t = I.normal(7, 40)
    loss, g = M.loss_and_grad(rng_p, norm, x, t, bf16=False)
    h = 1e-6
    idx = list(range(0, 320, 37)) + [320, 333, 384 + 5, 384 + 64 * 33, 4480 + 3, 4544 + 10, 4608]
    for i in idx:
        e = np.zeros_like(rng_p); e[i] = h
        fp = M.loss_and_grad(rng_p + e, norm, x, t, bf16=False)[0]
        fm = M.loss_and_grad(rng_p - e, norm, x, t, bf16=False)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_reference_first_step():
    """First bias-corrected Adam step moves every parameter by lr * sign(g)
    (up to eps)."""
    p = np.zeros(10)
    g = np.linspace(-1, 1, 10) + 0.05
    p1, m, v = M.adam_step(p, np.zeros(10), np.zeros(10), g, 1, lr=1e-3)
    np.testing.assert_allclose(p1, -1e-3 * np.sign(g), rtol=1e-6)


def test_features_match_conservative_scaling():
    """features depend on D/E and |S|/E only: scaling the state leaves them
    unchanged; the target log(p/E) likewise."""
    cons, p = I.srhd_training_pairs(9, 100)
    f1 = M.features(cons)
    f2 = M.features(cons * 7.5)
    np.testing.assert_allclose(f1[:, :4], f2[:, :4], rtol=1e-13, atol=1e-13)
    # the internal-energy feature cancels O(E^2) terms down to O(rho eps E):
    # scaling changes its rounding, not its value
    np.testing.assert_allclose(f1[:, 4], f2[:, 4], rtol=0, atol=1e-8)


def test_standardise_is_the_quotient_up_to_rounding():
    """(x - m) * rn(1/s) against (x - m) / s: equal when s is a power of two
    (exact reciprocal) and within 1.5 binary32 ulp otherwise (the product of
    a half-ulp reciprocal error and a half-ulp product rounding)."""
    x = I.normal(21, 4000).reshape(800, 5) * 3.0
    norm = np.array([0.5, -1.0, 0.25, 2.0, -0.75, 2.0, 0.5, 4.0, 1.0, 0.125, 0.0, 1.0], np.float32)
    z = M.standardise(x, norm, bf16=False)
    x32 = x.astype(np.float32)
    q = ((x32 - norm[:5]) / norm[5:10]).astype(np.float64)
    np.testing.assert_array_equal(z, q)
    norm2 = norm.copy()
    norm2[5:10] = [0.3, 1.7, 2.9, 0.77, 5.3]
    z2 = M.standardise(x, norm2, bf16=False)
    q2 = ((x32 - norm2[:5]) / norm2[5:10]).astype(np.float32)
    ulp = np.spacing(np.abs(q2)).astype(np.float64)
    assert np.all(np.abs(z2 - q2.astype(np.float64)) <= 1.5 * ulp)


def test_training_target_closed_form():
    """log(p/E) of a cell at rest: tau = rho eps, E = rho (1 + eps) and
    p = (Gamma - 1) rho eps, so p/E = (Gamma - 1) eps / (1 + eps)."""
    rho = np.array([0.3, 2.0, 7.0])
    eps = np.array([0.01, 0.5, 9.0])
    z = np.zeros(3)
    cons, p = I.srhd_prim_to_cons(rho, z, z, z, eps, 5 / 3)
    t = M.target(cons, p)
    np.testing.assert_allclose(t, np.log((2 / 3) * eps / (1 + eps)).astype(np.float32), rtol=1e-6)


def test_fit_norm_closed_form():
    """mean and sample standard deviation (divisor n - 1) of 1..n are
    (n + 1)/2 and sqrt(n (n + 1) / 12); a constant column takes the 1e-6
    floor (features only)."""
    n = 1001
    v = np.arange(1, n + 1, dtype=np.float64)
    x = np.stack([v, 2 * v, -v, np.full(n, 3.0), v / 4], axis=1)
    norm = M.fit_norm(x, v)
    s = math.sqrt(n * (n + 1) / 12.0)
    np.testing.assert_allclose(norm[:5], np.float32([(n + 1) / 2, n + 1, -(n + 1) / 2, 3.0, (n + 1) / 8]), rtol=1e-7)
    np.testing.assert_allclose(norm[5:10], np.float32([s, 2 * s, s, 1e-6, s / 4]), rtol=1e-6)
    np.testing.assert_allclose(norm[10:], np.float32([(n + 1) / 2, s]), rtol=1e-7)
    t = M.standardise_target(v, norm)
    np.testing.assert_allclose(t[[0, n // 2, n - 1]], [-(n - 1) / 2 / s, 0.0, (n - 1) / 2 / s], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 1000, 4096, 12345])
def test_training_permutation_is_a_seeded_bijection(n):
    """the epoch permutation of the training rows covers [0, n) exactly once,
    depends on seed and epoch, and is reproducible"""
    a = I.feistel_permutation(2024, 0, n)
    np.testing.assert_array_equal(np.sort(a), np.arange(n))
    np.testing.assert_array_equal(a, I.feistel_permutation(2024, 0, n))
    if n >= 1000:
        assert np.mean(a != I.feistel_permutation(2024, 1, n)) > 0.99
        assert np.mean(a != I.feistel_permutation(7, 0, n)) > 0.99
        assert abs(np.corrcoef(np.arange(n), a)[0, 1]) < 0.1
