"""GPU checks of the learned-guess network: matrix-core forward pass and the
training kernels' gradients against the oracle, training progress, and what
the trained guess buys the con2prim Newton iteration."""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I
from paper_2608_19273_amd import mlp_train

from gpu_helpers import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu


def random_net(seed=11):
    p = (I.normal(seed, M.NPARAM) * 0.3).astype(np.float32)
    norm = np.array([-1.0, 0.4, -0.8, -1.5, 0.3, 1.2, 0.3, 0.9, 1.1, 0.25, -3.0, 2.5], np.float32)
    return p, norm


def test_features_match_oracle():
    announce("mlp features")
    torch = need_gpu()
    cons, _ = I.srhd_training_pairs(4, 5000)
    x = pb.pb_mlp_features(torch.from_numpy(cons).cuda()).cpu().numpy()
    np.testing.assert_allclose(x, M.features(cons).astype(np.float32), rtol=2e-6, atol=2e-6)


def test_forward_matches_oracle():
    """Both sides round the same values to bf16 at the same points; they
    differ by the FP32 (matrix cores) against FP64 (oracle) accumulation.
    Most rows agree to the FP32 accumulation bound of the last layer, (K+1)
    2^-24 sum |terms|; a hidden activation that lies within that accumulation
    error of a bf16 rounding midpoint may round one bf16 ulp apart, so every
    row must lie within the bound of one-ulp flips of its activations
    (propagated through the weights), and such rows must stay a small
    minority."""
    announce("mlp forward")
    torch = need_gpu()
    p, norm = random_net()
    net = pb.Mlp(p, norm)
    x = (I.normal(12, 20000 * 5).reshape(20000, 5) * np.array([1.0, 0.2, 0.8, 1.0, 0.2]) + norm[:5]).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yo, (xb, h1, h2, W1, W2, w3) = M.forward(p, norm, x, keep=True)
    _, _, _, _, _, b3 = M.unpack(p)
    u = 2.0 ** -24
    e3 = 65 * u * (np.abs(h2) @ np.abs(w3) + abs(b3))
    ulp = lambda h: np.exp2(np.floor(np.log2(np.where(h > 0, h, 1.0))) - 7) * (h > 0)
    flip = ulp(h2) @ np.abs(w3) + (ulp(h1) @ np.abs(W2).T) @ np.abs(w3)
    d = np.abs(y - yo)
    tight = d <= e3
    assert tight.mean() >= 0.8, tight.mean()
    assert np.all(d <= e3 + flip), np.max(d / (e3 + flip))
    net.close()


def test_prepare_matches_oracle():
    """pb_mlp_prepare: raw features within a few binary32 ulp of the oracle's
    FP64 features (FP32 ratios and logarithms on the GPU), targets
    binary32(log(p/E)) within one ulp (FP64 logarithms of both sides)"""
    announce("mlp prepare")
    torch = need_gpu()
    cons, p = I.srhd_training_pairs(31, 50000)
    x, y = pb.pb_mlp_prepare(torch.from_numpy(cons).cuda(), torch.from_numpy(p).cuda())
    np.testing.assert_allclose(x.cpu().numpy(), M.features(cons).astype(np.float32), rtol=2e-6, atol=2e-6)
    yo = M.target(cons, p)
    yg = y.cpu().numpy()
    assert np.all(np.abs(yg - yo) <= np.spacing(np.abs(yo)))


def test_fit_norm_and_standardise_match_oracle():
    """pb_mlp_fit_norm: means and standard deviations (FP64 sums in the
    library's fixed order against numpy's) within one binary32 ulp; the
    standardised target then bitwise equal to the oracle's with the same
    statistics"""
    announce("mlp fit_norm / standardise")
    torch = need_gpu()
    cons, p = I.srhd_training_pairs(32, 300001)
    x, y = pb.pb_mlp_prepare(torch.from_numpy(cons).cuda(), torch.from_numpy(p).cuda())
    net = pb.Mlp(*random_net(3))
    net.fit_norm(x, y)
    _, ng = net.get_params()
    no = M.fit_norm(x.cpu().numpy(), y.cpu().numpy())
    assert np.all(np.abs(ng - no) <= np.spacing(np.abs(no))), (ng, no)
    t = net.standardise_target(y).cpu().numpy()
    np.testing.assert_array_equal(t, M.standardise_target(y.cpu().numpy(), ng))
    net.close()


@pytest.mark.parametrize("n", [1, 7, 4096, 100003, 1 << 22])
def test_permutation_matches_generator(n):
    """the library's epoch permutation is bit for bit the one the input
    generator defines, for sizes with and without cycle walking"""
    announce(f"mlp permutation n={n}")
    need_gpu()
    for seed, epoch in ((2024, 0), (2024, 3), (5, 11)):
        g = pb.pb_mlp_permutation(seed, epoch, n).cpu().numpy()
        np.testing.assert_array_equal(g, I.feistel_permutation(seed, epoch, n))


def test_train_epoch_equals_gathered_steps():
    """pb_mlp_train_epoch (rows gathered inside the kernel through the epoch
    permutation, cosine learning rate) gives bit for bit the parameters and
    losses of pb_mlp_train_step calls on batches gathered on the host with
    the generator's permutation and the same schedule"""
    announce("mlp train_epoch")
    torch = need_gpu()
    import math
    n, batch, seed, lr = 5000, 1024, 99, np.float32(3e-3)
    x = torch.from_numpy((I.normal(40, n * 5).reshape(n, 5) * 0.8 + random_net()[1][:5]).astype(np.float32)).cuda()
    t = torch.from_numpy(I.normal(41, n).astype(np.float32)).cuda()
    p0, norm = random_net(42)
    A = pb.Mlp(p0, norm)
    Bn = pb.Mlp(p0, norm)
    spe = n // batch
    total = 2 * spe
    ls = torch.zeros(2, dtype=torch.float64, device="cuda")
    ref = np.zeros(2)
    for ep in range(2):
        A.train_epoch(x, t, batch, seed, ep, float(lr), ep * spe, total, loss_sum=ls[ep:])
        perm = torch.from_numpy(I.feistel_permutation(seed, ep, n)).cuda()
        for b in range(spe):
            step = ep * spe + b + 1
            lr_t = float(np.float32(0.5 * float(lr) * (1.0 + math.cos(math.pi * (step - 1) / total))))
            idx = perm[b * batch:(b + 1) * batch]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            Bn.train_step(xb, tb, lr_t, step, loss=loss)
            ref[ep] += float(loss.item())
    pa, _ = A.get_params()
    pbp, _ = Bn.get_params()
    np.testing.assert_array_equal(pa, pbp)
    np.testing.assert_allclose(ls.cpu().numpy(), ref, rtol=1e-12)
    A.close()
    Bn.close()


def test_gradient_matches_oracle():
    announce("mlp gradient")
    torch = need_gpu()
    p, norm = random_net(13)
    net = pb.Mlp(p, norm)
    n = 8192
    x = (I.normal(14, n * 5).reshape(n, 5) * 0.8 + norm[:5]).astype(np.float32)
    t = I.normal(15, n).astype(np.float32)
    g, loss = net.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    lo, go = M.loss_and_grad(p, norm, x, t)
    assert abs(loss.item() - lo) <= 1e-4 * lo
    offs = [0, 320, 384, 4480, 4544, 4608, 4609]
    for a, b_ in zip(offs[:-1], offs[1:]):
        num = np.linalg.norm(g[a:b_] - go[a:b_])
        den = np.linalg.norm(go[a:b_])
        assert num <= 1e-2 * den + 1e-7, (a, num / den)
    # one Adam step moves the parameters as the reference does
    net.train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), 1e-3, 1)
    p1, _ = net.get_params()
    pr, _, _ = M.adam_step(p.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM), g, 1, lr=1e-3)
    np.testing.assert_allclose(p1, pr, rtol=0, atol=2e-6)
    net.close()


def test_adam_steps_match_oracle():
    """Eight pb_mlp_train_step calls on one batch (bias correction at t = 1..8):
    before each call the library's gradient of the current parameters is
    taken, and the oracle's Adam, fed with those gradients and carrying its
    own moments in float64, must give the parameters the library holds after
    the call."""
    announce("mlp adam steps")
    torch = need_gpu()
    p, norm = random_net(17)
    net = pb.Mlp(p, norm)
    n = 4096
    x = torch.from_numpy((I.normal(18, n * 5).reshape(n, 5) * 0.8 + norm[:5]).astype(np.float32)).cuda()
    t = torch.from_numpy(I.normal(19, n).astype(np.float32)).cuda()
    cur = p.astype(np.float64)
    m = np.zeros(M.NPARAM)
    v = np.zeros(M.NPARAM)
    lr = 2e-3
    for step in range(1, 9):
        g, _ = net.grad(x, t)
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(x, t, lr, step)
        cur, m, v = M.adam_step(cur, m, v, g, step, lr=lr)
        got, _ = net.get_params()
        np.testing.assert_allclose(got, cur, rtol=0, atol=5e-6, err_msg=f"step {step}")
        cur = got.astype(np.float64)
    net.close()


@pytest.fixture(scope="module")
def trained():
    need_gpu()
    net, hist = mlp_train.train(n_pairs=1 << 18, epochs=10, batch=1024, lr=3e-3, seed=5)
    return net, hist


def test_training_reduces_loss(trained):
    announce("mlp training")
    net, hist = trained
    L = hist["epoch_loss"]
    assert L[-1] < 0.05 * L[0] and L[-1] < 5e-3, L


def test_learned_guess_saves_iterations(trained):
    """Held-out states (other seed): the learned start needs fewer Newton
    updates than the plain start (mean and per-wave maximum) and converges to
    the same pressures (within the conditioning of the problem)."""
    announce("learned guess gain")
    torch = need_gpu()
    net, _ = trained
    n = 1 << 16
    cons, p = I.srhd_training_pairs(999, n)
    c = torch.from_numpy(cons).cuda()
    out = {}
    for guess in ("plain", "learned"):
        prim = torch.empty((5, n), dtype=torch.float64, device="cuda")
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        pb.con2prim(c, prim, 5 / 3, 1e-12, 50, guess=guess, mlp=net if guess == "learned" else None,
                    iters=it, status=st)
        out[guess] = (prim[4].cpu().numpy(), it.cpu().numpy(), st.cpu().numpy())
    pp, ip, sp = out["plain"]
    pl, il, sl = out["learned"]
    assert np.all(sp == 0) and np.all(sl == 0)
    assert il.mean() < 0.7 * ip.mean(), (il.mean(), ip.mean())
    wave_max = lambda a: a.reshape(-1, 64).max(axis=1).mean()
    assert wave_max(il) < wave_max(ip)
    rho, vx, vy, vz, pr = oracle.con2prim(cons)[0]
    W2 = 1.0 / (1.0 - (vx * vx + vy * vy + vz * vz))
    eps = pr / ((5 / 3 - 1) * rho)
    bound = np.maximum(1e-12, 8 * 2.2e-16 * W2 / eps)
    assert np.all(np.abs(pl - pp) / pp <= 2 * bound)


def test_learned_srhd_step_parity(trained):
    """The SRHD step with the learned guess matches the plain-guess oracle."""
    announce("learned srhd step")
    net, _ = trained
    b = I.config3(grid=(2, 2, 2), seed=41)
    o, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=2)
    B = pb.PatchBatch(b)
    B.set_c2p_guess("learned", net)
    B.fv_rusanov_step(cfl=0.4, n_steps=2)
    g = B.download()
    st = B.stats()
    B.close()
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    assert st["c2p_failures"] == 0
