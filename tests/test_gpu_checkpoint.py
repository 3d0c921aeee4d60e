"""Checkpoint and resume: the state lives in caller-owned buffers, so a
checkpoint is the downloaded state (plus the network's parameters for the
learned guess).  A run split into two calls on two batches, the second one
created from the first one's downloaded state, must equal the uninterrupted
run bitwise: every kernel is deterministic and dt comes from the state."""
import numpy as np
import pytest

import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

from gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


def split_run(b, step, n1, n2, storage="fp64", setup=None):
    """(uninterrupted n1 + n2 steps, n1 steps then resume from the downloaded
    state for n2 steps); `step(B, n)` advances a batch by n steps"""
    need_gpu()
    B = pb.PatchBatch(b, storage=storage)
    if setup:
        setup(B)
    step(B, n1 + n2)
    whole = B.download()
    B.close()
    B = pb.PatchBatch(b, storage=storage)
    if setup:
        setup(B)
    step(B, n1)
    ckpt = B.download()
    B.close()
    B = pb.PatchBatch(b, storage=storage, state=ckpt)
    if setup:
        setup(B)
    step(B, n2)
    resumed = B.download()
    B.close()
    return whole, resumed


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_fv_euler_resume_bitwise(storage):
    announce(f"checkpoint fv euler {storage}")
    b = I.config1(grid=(4, 4, 2))
    whole, resumed = split_run(b, lambda B, n: B.fv_rusanov_step(cfl=0.4, n_steps=n), 5, 5, storage)
    np.testing.assert_array_equal(whole, resumed)


def test_fd_euler_resume_bitwise():
    announce("checkpoint fd euler")
    b = I.config1(grid=(2, 2, 2), halo=3)
    whole, resumed = split_run(b, lambda B, n: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n), 3, 2)
    np.testing.assert_array_equal(whole, resumed)


def test_linear_system_resume_bitwise():
    announce("checkpoint linear system")
    b = I.config2(subset=I.config2_subset(n_per_size=(2, 2, 2)))
    whole, resumed = split_run(b, lambda B, n: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n), 2, 2)
    np.testing.assert_array_equal(whole, resumed)


def test_srhd_resume():
    """Plain and learned guesses hold no history, so a resumed run is bitwise
    the uninterrupted one; the network is checkpointed as its parameters and
    normalisation and rebuilt.  The warm start's previous pressure lives in
    the workspace, not in the state: the resumed run's first step starts from
    the plain guess, and Newton converges to the same pressures to the
    tolerance, so the states agree to roundoff only."""
    announce("checkpoint srhd")
    from paper_2608_19273_amd import mlp_train
    net, _ = mlp_train.train(n_pairs=1 << 16, epochs=2, batch=1024, lr=3e-3, seed=9)
    params, norm = net.get_params()
    net2 = pb.Mlp(params, norm)
    b = I.config3(grid=(2, 2, 2))
    step = lambda B, n: B.fv_rusanov_step(cfl=0.4, n_steps=n)
    whole, resumed = split_run(b, step, 2, 2)
    np.testing.assert_array_equal(whole, resumed)
    whole, _ = split_run(b, step, 2, 2, setup=lambda B: B.set_c2p_guess("learned", net))
    _, resumed = split_run(b, step, 2, 2, setup=lambda B: B.set_c2p_guess("learned", net2))
    np.testing.assert_array_equal(whole, resumed)
    whole, resumed = split_run(b, step, 2, 2, setup=lambda B: B.set_c2p_guess("warm"))
    scale = np.abs(whole).max()
    assert np.max(np.abs(whole - resumed)) <= 1e-12 * scale
    net.close()
    net2.close()
