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
    announce("mlp forward")
    torch = need_gpu()
    p, norm = random_net()
    net = pb.Mlp(p, norm)
    x = (I.normal(12, 20000 * 5).reshape(20000, 5) * np.array([1.0, 0.2, 0.8, 1.0, 0.2]) + norm[:5]).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = M.forward(p, norm, x)
    d = np.abs(y - yo)
    assert np.quantile(d, 0.999) <= 1e-3 * (1 + np.abs(yo).max()), np.quantile(d, 0.999)
    assert d.max() <= 2e-2 * (1 + np.abs(yo).max())
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
