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


def _bf16_clear(v, err):
    """True where a binary32 value v lies farther than `err` from the nearest
    bf16 rounding midpoint (so any value within err of v rounds to the same
    bf16 number); zeros (ReLU-clipped) are clear"""
    v32 = np.asarray(v, np.float32)
    u = v32.view(np.uint32).astype(np.int64)
    frac = np.abs((u & 0xFFFF) - 0x8000) / 65536.0          # in bf16 ulps
    a = np.abs(v32.astype(np.float64))
    ulp = np.exp2(np.floor(np.log2(np.where(a > 0, a, 1.0))) - 7)
    return (a == 0) | (frac * ulp > err)


def test_forward_matches_oracle():
    """Per row: where every bf16 rounding of the hidden activations lies
    farther from a rounding midpoint than twice the FP32 accumulation bound of
    its dot product ((K+1) 2^-24 sum |terms|), both sides round identically and
    the outputs must agree to the FP32 accumulation bound of the last layer;
    rows with an activation near a midpoint may flip one bf16 ulp and are
    bounded in number."""
    announce("mlp forward")
    torch = need_gpu()
    p, norm = random_net()
    net = pb.Mlp(p, norm)
    x = (I.normal(12, 20000 * 5).reshape(20000, 5) * np.array([1.0, 0.2, 0.8, 1.0, 0.2]) + norm[:5]).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yo, (xb, h1, h2, W1, W2, w3) = M.forward(p, norm, x, keep=True)
    _, b1, _, b2, _, b3 = M.unpack(p)
    u = 2.0 ** -24
    a1 = xb @ W1.T + b1
    e1 = 6 * u * (np.abs(xb) @ np.abs(W1).T + np.abs(b1))
    a2 = h1 @ W2.T + b2
    e2 = 65 * u * (np.abs(h1) @ np.abs(W2).T + np.abs(b2))
    clear = (_bf16_clear(np.maximum(a1, 0), 2 * e1) | (a1 + e1 < 0)).all(axis=1) & \
            (_bf16_clear(np.maximum(a2, 0), 2 * e2) | (a2 + e2 < 0)).all(axis=1)
    d = np.abs(y - yo)
    e3 = 65 * u * (np.abs(h2) @ np.abs(w3) + abs(b3))
    assert clear.mean() > 0.5, clear.mean()
    assert np.all(d[clear] <= e3[clear]), (d[clear] / e3[clear]).max()
    assert np.all(d <= 2e-2 * (1 + np.abs(yo).max()))
    net.close()


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
