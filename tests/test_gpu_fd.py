"""GPU parity of the FD4 + KO6 + RK4 stage kernels (FP64 matrix cores for
the B.grad Q product) against the oracle and the plane-wave closed form."""
import numpy as np
import pytest

import oracle
import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

from gpu_helpers import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu


def run_fd(batch, n_steps=1, cfl=0.5, dt_fixed=0.0, sigma=0.1, rk=4, use_graph=False):
    need_gpu()
    B = pb.PatchBatch(batch)
    dt = B.fd_ko_step(cfl=cfl, dt_fixed=dt_fixed, sigma_ko=sigma, rk_stages=rk, n_steps=n_steps,
                      use_graph=use_graph, want_dt=True)
    out = B.download()
    B.close()
    return out, dt


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_wave_closed_form(axis):
    """One self-periodic 16^3 patch, N = 7, plane wave on an eigenvector of
    B_axis: R(z)^n times the initial wave, z from the D4/KO6 symbols."""
    announce(f"fd plane wave axis {axis}")
    N, p = 7, 16
    Bs, rhos = I.linsym_matrices(8, N)
    b = I.Batch(dim=3, p=np.array([p], np.int32), dx=np.array([1.0 / p]), nbr=I.self_periodic(1, 3), halo=3,
                pde="linsym", params=I.linsym_params(Bs, rhos), n_unknowns=N, state=np.zeros(N * p ** 3))
    lamv, vecs = np.linalg.eigh(Bs[axis])
    lam, r = lamv[2], vecs[:, 2]
    theta = 2 * np.pi * 3 / p
    prof = np.cos(theta * np.arange(p))
    shape = [1, 1, 1]
    shape[2 - axis] = p
    g = r[:, None, None, None] * prof.reshape(shape)[None] * np.ones((N, p, p, p))
    b.state = g.reshape(-1).copy()
    n = 3
    out, dt = run_fd(b, n_steps=n, sigma=0.1)
    dx = 1.0 / p
    z = dt * (-1j * lam * (8 * np.sin(theta) - np.sin(2 * theta)) / (6 * dx) - 0.1 * np.sin(theta / 2) ** 6 / dx)
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    ex = np.real(R ** n * np.exp(1j * theta * np.arange(p)))
    exg = r[:, None, None, None] * ex.reshape(shape)[None] * np.ones((N, p, p, p))
    np.testing.assert_allclose(out.reshape(N, p, p, p), exg, rtol=0, atol=1e-13)


def test_config2_subset_parity():
    """48 seeded patches of the full uneven batch (16 each of 4^3, 8^3,
    16^3), N = 58, sigma 0.1, CFL 0.5, ten RK4 steps (the step count read
    for the configuration), through the graph-captured launches the benchmark
    replays."""
    announce("fd config2 subset, 10 steps")
    sel = I.config2_subset()
    b = I.config2(subset=sel)
    o, dts = oracle.fd_step(b, cfl=0.5, sigma=0.1, n_steps=10)
    g, dt = run_fd(b, n_steps=10, use_graph=True)
    assert abs(dt - dts[-1]) <= 1e-15 * dts[-1]
    err = rel_err(b, g, o)
    assert np.all(err <= 1e-12), err.max()


def test_forward_euler_stage_and_graph():
    announce("fd rk1 / graph")
    b = I.config2(n_patches=6, N=20, sizes=np.array([8, 4, 16, 8, 4, 8], np.int32))
    o, _ = oracle.fd_step(b, cfl=0.5, sigma=0.05, rk_stages=1, n_steps=2)
    g, _ = run_fd(b, n_steps=2, sigma=0.05, rk=1)
    assert np.all(rel_err(b, g, o) <= 1e-12)
    o4, _ = oracle.fd_step(b, cfl=0.5, sigma=0.05, n_steps=3)
    g4, _ = run_fd(b, n_steps=3, sigma=0.05, use_graph=True)
    assert np.all(rel_err(b, g4, o4) <= 1e-12)


def test_batch_permutation_invariance():
    """Independent patches: reversing the batch order permutes the
    per-patch results bitwise."""
    announce("fd permutation")
    b = I.config2(n_patches=8, N=58, sizes=np.array([4, 8, 16, 4, 8, 4, 16, 8], np.int32))
    g, _ = run_fd(b)
    perm = np.arange(8)[::-1]
    bp = b.copy()
    bp.p = b.p[perm]
    bp.dx = b.dx[perm]
    bp.state = np.concatenate([b.patch_view(b.state, k).reshape(-1) for k in perm])
    gp, _ = run_fd(bp)
    for j, k in enumerate(perm):
        np.testing.assert_array_equal(bp.patch_view(gp, j), b.patch_view(g, k))


def test_energy_nonincreasing_gpu():
    announce("fd energy")
    b = I.config2(n_patches=4, N=58, sizes=np.array([8, 16, 4, 8], np.int32))
    b.state = I.uniform(3, b.state.size, -1, 1)
    g, _ = run_fd(b, n_steps=3, sigma=0.1)
    assert np.sum(g ** 2) < np.sum(b.state ** 2)


@pytest.mark.slow
def test_config2_full_size_sampled_patches():
    """The full 4096-patch batch in the benchmark's launch configuration; the
    patches are independent, so the oracle recomputes a seeded sample of 12
    (4 per size) on their own with the same dt."""
    announce("fd config2 full size")
    b = I.config2()
    g, dt = run_fd(b, n_steps=1)
    sizes = b.p
    rng = I.splitmix64(123, 12)
    pick = []
    for j, ps in enumerate((4, 8, 16)):
        where = np.nonzero(sizes == ps)[0]
        pick += [int(where[int(v % np.uint64(len(where)))]) for v in rng[4 * j:4 * j + 4]]
    sub = I.config2(subset=pick, sizes=sizes)
    o, _ = oracle.fd_step(sub, dt_fixed=dt, sigma=0.1, n_steps=1)
    for j, k in enumerate(pick):
        ref = sub.patch_view(o, j)
        got = b.patch_view(g, k)
        err = np.max(np.abs(got - ref), axis=(1, 2, 3)) / np.max(np.abs(ref), axis=(1, 2, 3))
        assert np.all(err <= 1e-12), (k, err.max())


@pytest.mark.parametrize("N", [1, 5, 8, 13, 20, 29, 33, 47, 53, 58, 60])
def test_wave_specialised_kernel_matches(N):
    """The wave-specialised stage kernel (the default) against the oracle and,
    bitwise, against the kernel in which every wave does every phase, for
    every number of 8-unknown chunks (1..8, N not a multiple of 4 or 8
    included), with and without the XCD-grouped tile order, on 5 uneven
    patches (fewer tiles than CUs, so most
    work-groups own one tile and the pipeline runs past its last step)."""
    announce(f"fd wave-specialised N={N}")
    need_gpu()
    b = I.config2(n_patches=5, N=N, sizes=np.array([8, 4, 16, 4, 8], np.int32))
    out = {}
    for ws, remap in ((1, 1), (1, 0), (0, 1)):
        B = pb.PatchBatch(b)
        B.set_tuning(fd_ws=ws, fd_xcd_remap=remap)
        assert B.get_tuning()["fd_ws"] == ws
        B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
        B.fd_ko_step(cfl=0.5, dt_fixed=1e-3, sigma_ko=0.05, rk_stages=1, n_steps=1)
        out[(ws, remap)] = B.download()
        B.close()
    np.testing.assert_array_equal(out[(1, 1)], out[(0, 1)])
    np.testing.assert_array_equal(out[(1, 0)], out[(0, 1)])
    out[1] = out[(1, 1)]
    o, _ = oracle.fd_step(b, cfl=0.5, sigma=0.1, n_steps=2)
    b2 = b.copy()
    b2.state = o
    o2, _ = oracle.fd_step(b2, dt_fixed=1e-3, sigma=0.05, rk_stages=1, n_steps=1)
    assert np.all(rel_err(b, out[1], o2) <= 1e-12)


@pytest.mark.parametrize("N", [1, 3, 4, 5, 8, 13, 20, 29, 33, 47, 53, 57, 58, 60])
def test_tile_kernel_matches(N):
    """The one-wave-per-tile stage kernel (fd_ws = 2) against the oracle and,
    to roundoff (it adds the K steps in another order), against the
    wave-specialised kernel, for every count of 4-unknown chunks (N = 1..60,
    ragged last chunks), both tile orders, RK4 with CFL dt and a fixed-dt
    forward Euler step, on 5 uneven patches."""
    announce(f"fd tile kernel N={N}")
    need_gpu()
    b = I.config2(n_patches=5, N=N, sizes=np.array([8, 4, 16, 4, 8], np.int32))
    out = {}
    for ws, remap in ((2, 1), (2, 0), (1, 1)):
        B = pb.PatchBatch(b)
        B.set_tuning(fd_ws=ws, fd_xcd_remap=remap)
        assert B.get_tuning()["fd_ws"] == ws
        B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
        B.fd_ko_step(cfl=0.5, dt_fixed=1e-3, sigma_ko=0.05, rk_stages=1, n_steps=1)
        out[(ws, remap)] = B.download()
        B.close()
    np.testing.assert_array_equal(out[(2, 1)], out[(2, 0)])
    assert np.all(rel_err(b, out[(2, 1)], out[(1, 1)]) <= 1e-14)
    o, _ = oracle.fd_step(b, cfl=0.5, sigma=0.1, n_steps=2)
    b2 = b.copy()
    b2.state = o
    o2, _ = oracle.fd_step(b2, dt_fixed=1e-3, sigma=0.05, rk_stages=1, n_steps=1)
    assert np.all(rel_err(b, out[(2, 1)], o2) <= 1e-12)


def test_tile_kernel_config2_subset():
    """The 48-patch subset of the uneven 58-unknown batch, 10 graph-replayed
    RK4 steps with the one-wave-per-tile kernel, against the oracle."""
    announce("fd tile kernel config2 subset, 10 steps")
    need_gpu()
    b = I.config2(subset=I.config2_subset())
    o, dts = oracle.fd_step(b, cfl=0.5, sigma=0.1, n_steps=10)
    B = pb.PatchBatch(b)
    B.set_tuning(fd_ws=2, fd_xcd_remap=1)
    dt = B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=10, use_graph=True, want_dt=True)
    g = B.download()
    B.close()
    assert abs(dt - dts[-1]) <= 1e-15 * dts[-1]
    assert np.all(rel_err(b, g, o) <= 1e-12)


def test_graph_replays_match_eager():
    """Three steps captured in a HIP graph and replayed three times, with the
    program's own eager work and synchronisations between the replays: every
    replay equals the same steps run eagerly, bitwise (wave-specialised
    kernel, uneven patches, N = 58; the eager steps are held to the oracle by
    the parity tests above)."""
    announce("fd graph replays")
    torch = need_gpu()
    b = I.config2(n_patches=6, N=58, sizes=np.array([16, 4, 8, 8, 4, 16], np.int32))
    eager = pb.PatchBatch(b)
    graph = pb.PatchBatch(b)
    for rep in range(3):
        eager.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=3)
        graph.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=3, use_graph=True)
        torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(graph.download(), eager.download())
    eager.close()
    graph.close()
