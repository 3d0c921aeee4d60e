"""GPU parity of the fused Rusanov FV step (HIP, through the C ABI) against
the CPU oracle, plus the invariants checked on the GPU path itself."""
import numpy as np
import pytest

import oracle
import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

from gpu_helpers import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu


def run_gpu(batch, storage="fp64", n_steps=1, cfl=0.4, dt_fixed=0.0, use_graph=False, tuning=None, poison=False):
    torch = need_gpu()
    B = pb.PatchBatch(batch, storage=storage)
    if poison:
        B.bufs[1].fill_(float("nan"))
    if tuning:
        B.set_tuning(**tuning)
    dt = B.fv_rusanov_step(cfl=cfl, dt_fixed=dt_fixed, n_steps=n_steps, use_graph=use_graph, want_dt=True)
    out = B.download()
    st = B.stats()
    B.close()
    return out, dt, st


def test_config0_parity():
    """2D Euler entropy wave, 64x64 as 8x8 patches of 8^2, CFL 0.4, 10 steps."""
    announce("config0 parity")
    b = I.config0()
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=10)
    g, dt, st = run_gpu(b, n_steps=10)
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    assert abs(dt - dts[-1]) <= 1e-14 * dts[-1]
    assert st["nonfinite_units"] == 0


@pytest.mark.parametrize("slab", [0, 1, 5, 16])
def test_euler3d_parity_and_slab_invariance(slab):
    """3D Euler, smooth random IC on 4x4x2 patches of 16^3, 5 steps.  Every
    z-slab decomposition agrees to roundoff (the z face at a slab boundary is
    evaluated by both slabs, in differently inlined code), and a repeated run
    of one decomposition is bitwise identical."""
    announce(f"euler3d slab={slab}")
    b = I.config1(grid=(4, 4, 2))
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=5)
    g, dt, _ = run_gpu(b, n_steps=5, tuning={"fv_slab": slab, "fv_xcd_remap": 1})
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    g0, _, _ = run_gpu(b, n_steps=5, tuning={"fv_slab": 0, "fv_xcd_remap": 0})
    assert np.all(rel_err(b, g, g0) <= 1e-14)
    g1, _, _ = run_gpu(b, n_steps=5, tuning={"fv_slab": slab, "fv_xcd_remap": 1})
    np.testing.assert_array_equal(g, g1)


@pytest.mark.parametrize("grid,storage", [((4, 4, 2), "fp64"), ((8, 8, 4), "fp64"), ((8, 8, 4), "fp32"),
                                          ((16, 16, 3), "fp64")])
def test_euler3d_balanced_schedule(grid, storage):
    """The balanced plane schedule (one work-group per resident slot, each
    marching an equal run of the batch's planes across patch boundaries):
    32 patches (fewer planes than slots: one plane per work-group), 256
    patches (runs of 5-6 planes crossing patches) and 768 patches (16 planes
    per slot, runs starting mid-patch); against the oracle, against slab mode
    to roundoff, bitwise repeatable, both XCD orders, 2, 3 and 5
    work-groups per CU (5: more than fit at once, so a second round)."""
    announce(f"euler3d balanced schedule {grid} {storage}")
    b = I.config1(grid=grid)
    tol = 1e-12
    if storage == "fp32":
        b.state = b.state.astype(np.float32).astype(np.float64)
        tol = 1e-5
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=3, round_fp32=storage == "fp32")
    gs, _, _ = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_slab": 0, "fv_xcd_remap": 1})
    for wgs, remap in ((3, 1), (3, 0), (2, 1), (5, 1)):
        g, dt, st = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_persist": wgs, "fv_xcd_remap": remap})
        assert np.all(rel_err(b, g, o) <= tol), rel_err(b, g, o)
        assert np.all(rel_err(b, g, gs) <= (1e-14 if storage == "fp64" else 1e-6))
        assert abs(dt - dts[-1]) <= 1e-13 * dts[-1]
        assert st["nonfinite_units"] == 0
        g2, _, _ = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_persist": wgs, "fv_xcd_remap": remap})
        np.testing.assert_array_equal(g, g2)


def test_euler3d_fp32_storage():
    announce("euler3d fp32 storage")
    b = I.config1(grid=(4, 4, 2))
    b.state = b.state.astype(np.float32).astype(np.float64)
    o32, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=5, round_fp32=True)
    o64, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=5)
    g, _, _ = run_gpu(b, storage="fp32", n_steps=5)
    assert np.all(rel_err(b, g, o32) <= 1e-5), rel_err(b, g, o32)
    assert np.all(rel_err(b, g, o64) <= 1e-5), rel_err(b, g, o64)


@pytest.mark.parametrize("p,grid", [(1, (3, 2, 2)), (2, (3, 3, 2)), (3, (4, 3, 3)), (4, (3, 2, 1)),
                                    (5, (2, 2, 3)), (6, (3, 2, 2))])
def test_small_patch_kernel(p, grid):
    """3D batches of one p with p^3 <= 256 run the kernel that packs whole
    patches into a work-group (one thread per cell, halos staged in an LDS
    box); patch counts that are not a multiple of the group size leave a
    partly filled last work-group.  Three CFL steps, FP64 and FP32 storage."""
    announce(f"small patches p={p} grid={grid}")
    b = I.config1(grid=grid, p=p, seed=50 + p)
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=3)
    g, dt, st = run_gpu(b, n_steps=3)
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    assert abs(dt - dts[-1]) <= 1e-14 * dts[-1]
    assert st["nonfinite_units"] == 0
    b32 = b.copy()
    b32.state = b.state.astype(np.float32).astype(np.float64)
    o32, _, _ = oracle.fv_step(b32, cfl=0.4, n_steps=3, round_fp32=True)
    g32, _, _ = run_gpu(b32, storage="fp32", n_steps=3)
    assert np.all(rel_err(b32, g32, o32) <= 1e-5), rel_err(b32, g32, o32)


def test_small_patch_advection_exact_shift():
    """Advection at CFL 1 along each axis is an exact shift by one cell, also
    through the small-patch kernel's halo staging (3^3 patches, 2x2x2 grid)."""
    announce("small patches exact shift")
    for axis in range(3):
        a = [0.0, 0.0, 0.0]
        a[axis] = 1.0
        b = I.make_uniform_batch((2, 2, 2), 3, 1, "adv_f", a + [0.0], 1, 1.0 / 6)
        b.state = I.uniform(90 + axis, b.state.size, -1.0, 1.0)
        g, _, _ = run_gpu(b, n_steps=1, cfl=1.0)
        ref = b.to_global(b.state, (2, 2, 2))
        np.testing.assert_allclose(b.to_global(g, (2, 2, 2)), np.roll(ref, 1, axis=3 - axis), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,p,field,storage,dma", [(3, 8, "random", "fp64", 0), (3, 16, "shear", "fp64", 0),
                                                      (3, 16, "random", "fp64", 1), (3, 4, "random", "fp32", 0),
                                                      (3, 5, "random", "fp64", 0), (2, 8, "random", "fp64", 0)])
def test_material_parameters_advection(dim, p, field, storage, dma):
    """Advection by a velocity field held as material parameters (N = 1
    evolving, M = dim carried) through the plane kernel (8^3, 16^3; also the
    DMA-fed one), the small-patch kernel (4^3, 5^3) and the 2D kernel: the
    field comes back bitwise, q matches the oracle, dt comes from the field."""
    announce(f"adv_var dim={dim} p={p} {field} {storage} dma={dma}")
    grid = (2, 2, 2) if dim == 3 else (3, 2)
    b = I.adv_var_batch(grid, p, kappa=0.1, field=field, seed=80 + p)
    f32 = storage == "fp32"
    if f32:
        b.state = b.state.astype(np.float32).astype(np.float64)
    o, dts, _ = oracle.fv_step(b, cfl=0.5, n_steps=4, round_fp32=f32)
    g, dt, st = run_gpu(b, storage=storage, n_steps=4, cfl=0.5, tuning={"fv_dma": dma} if dma else None)
    tol = 1e-5 if f32 else 1e-12
    assert rel_err(b, g, o)[0] <= tol, rel_err(b, g, o)
    for k in range(b.K):
        np.testing.assert_array_equal(b.patch_view(g, k)[1:], b.patch_view(b.state, k)[1:])
    assert abs(dt - dts[-1]) <= 1e-14 * dts[-1]
    assert st["nonfinite_units"] == 0


@pytest.mark.parametrize("form", ["adv_f", "adv_b"])
@pytest.mark.parametrize("dim", [2, 3])
def test_exact_shift_gpu(form, dim):
    """CFL 1 axis-aligned advection shifts by one cell per step (also across
    patch faces); parity with the oracle."""
    announce(f"exact shift {form} {dim}d")
    grid = (3, 2) if dim == 2 else (3, 2, 2)
    p = 8
    b = I.make_uniform_batch(grid, p, 1, form, [1.0, 0.0, 0.0, 0.0], 1, 1.0 / (grid[0] * p))
    b.state = I.uniform(3, b.total_cells, -1, 1)
    n = 5
    g, dt, _ = run_gpu(b, n_steps=n, cfl=1.0)
    g0 = b.to_global(b.state, grid)[0]
    np.testing.assert_allclose(b.to_global(g, grid)[0], np.roll(g0, n, axis=dim - 1), rtol=0, atol=1e-14)
    o, _, _ = oracle.fv_step(b, cfl=1.0, n_steps=n)
    assert np.all(rel_err(b, g, o) <= 1e-12)


@pytest.mark.parametrize("form", ["adv_f", "adv_b"])
def test_advection_source_any_cfl(form):
    announce(f"advection source {form}")
    b = I.make_uniform_batch((2, 3, 2), 6, 1, form, [0.7, -0.4, 0.3, 0.8], 1, 1.0 / 12)
    b.state = I.uniform(4, b.total_cells, -1, 1)
    o, dts, _ = oracle.fv_step(b, cfl=0.6, n_steps=4)
    g, dt, _ = run_gpu(b, n_steps=4, cfl=0.6)
    assert np.all(rel_err(b, g, o) <= 1e-12)


@pytest.mark.parametrize("grid,storage", [((4, 4, 2), "fp64"), ((8, 8, 3), "fp64"), ((8, 8, 4), "fp32"),
                                          ((16, 16, 3), "fp64")])
def test_euler3d_column_runs(grid, storage):
    """Column runs (each work-group marches a run of planes up a +z chain of
    patches, crossing patch tops without a restart): 32 patches (more slots
    than planes: runs of one plane), 192 patches in chains of 3 (one run of
    48 planes per chain at w = 1, runs of 12 crossing patch tops at w = 3),
    256 and 768 patches; against the oracle, against whole-patch slabs to
    roundoff, bitwise repeatable, both XCD orders."""
    announce(f"euler3d column runs {grid} {storage}")
    b = I.config1(grid=grid)
    tol = 1e-12
    if storage == "fp32":
        b.state = b.state.astype(np.float32).astype(np.float64)
        tol = 1e-5
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=3, round_fp32=storage == "fp32")
    gs, _, _ = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_slab": 0, "fv_xcd_remap": 1})
    for w, remap in ((3, 1), (3, 0), (2, 1), (1, 1), (8, 1)):
        g, dt, st = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_column": w, "fv_xcd_remap": remap})
        assert np.all(rel_err(b, g, o) <= tol), (w, remap, rel_err(b, g, o))
        assert np.all(rel_err(b, g, gs) <= (1e-14 if storage == "fp64" else 1e-6))
        assert abs(dt - dts[-1]) <= 1e-13 * dts[-1]
        assert st["nonfinite_units"] == 0
        g2, _, _ = run_gpu(b, storage=storage, n_steps=3, tuning={"fv_column": w, "fv_xcd_remap": remap})
        np.testing.assert_array_equal(g, g2)


@pytest.mark.parametrize("w", [1, 3])
def test_column_runs_open_chains_cover_every_cell(w):
    """8x8 columns of 3 patches of 16^3 whose bottom and top patches take
    their outer z halo from themselves (open +z chains, not cycles).  The
    output buffer starts as NaN, so a plane that no run marches stays NaN;
    one step, then three, against the oracle."""
    announce(f"column runs, open chains, w={w}")
    b = I.config1(grid=(8, 8, 3))
    layer, nz = 8 * 8, 3   # patch index = (z * ny + y) * nx + x
    nbr = b.nbr.copy()
    for k in range(b.K):
        if k // layer == 0:
            nbr[k, 4] = k
        if k // layer == nz - 1:
            nbr[k, 5] = k
    b.nbr = nbr
    for n_steps in (1, 3):
        o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=n_steps)
        g, dt, st = run_gpu(b, n_steps=n_steps, tuning={"fv_column": w}, poison=True)
        assert np.all(np.isfinite(g))
        assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
        assert abs(dt - dts[-1]) <= 1e-13 * dts[-1]
        assert st["nonfinite_units"] == 0


def test_ragged_patch_sizes():
    """Patches of p = 5 and p = 11 (not multiples of any tile) and p = 16 in
    one batch, each group periodic among itself."""
    announce("ragged patch sizes")
    ps = np.array([5, 5, 11, 16, 11], np.int32)
    nbr = np.array([[1, 1, 0, 0, 0, 0], [0, 0, 1, 1, 1, 1], [4, 4, 2, 2, 2, 2], [3] * 6, [2, 2, 4, 4, 4, 4]],
                   np.int32)
    K = len(ps)
    cells = int((ps.astype(np.int64) ** 3).sum())
    rho = I.uniform(5, cells, 0.8, 1.2)
    vel = [I.uniform(6 + i, cells, -0.3, 0.3) for i in range(3)]
    pr = I.uniform(9, cells, 0.8, 1.2)
    cons = np.stack(I.euler_prim_to_state(rho, vel, pr, 1.4))  # [5, cells]
    off = np.concatenate([[0], np.cumsum(ps.astype(np.int64) ** 3)])
    state = np.concatenate([cons[:, off[k]:off[k + 1]].reshape(-1) for k in range(K)])
    b = I.Batch(dim=3, p=ps, dx=1.0 / ps, nbr=nbr, halo=1, pde="euler", params=np.array([1.4]), n_unknowns=5,
                state=state)
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=3)
    g, dt, _ = run_gpu(b, n_steps=3, tuning={"fv_slab": 4, "fv_xcd_remap": 1})
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    # column runs: every patch is its own z cycle; 48 planes, so one run per plane
    g, dt, _ = run_gpu(b, n_steps=3, tuning={"fv_column": 3, "fv_xcd_remap": 1})
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)


def test_free_stream_conservation_determinism():
    announce("free stream / conservation / determinism")
    b = I.config0(n_patch=4, p=16)
    uni = b.copy()
    uni.state = b.from_global(np.stack([np.full((64, 64), v) for v in
                                        I.euler_prim_to_state(1.3, [0.4, -0.2], 0.9, 1.4)]), (4, 4))
    g, _, _ = run_gpu(uni, n_steps=4)
    np.testing.assert_array_equal(g, uni.state)
    rnd = b.copy()
    rnd.state = b.state * I.uniform(8, b.state.size, 0.9, 1.1)
    g1, _, _ = run_gpu(rnd, n_steps=6)
    g2, _, _ = run_gpu(rnd, n_steps=6, poison=True)
    np.testing.assert_array_equal(g1, g2)
    s0 = rnd.state.reshape(16, 4, -1).sum(axis=(0, 2))
    s1 = g1.reshape(16, 4, -1).sum(axis=(0, 2))
    np.testing.assert_allclose(s1, s0, rtol=1e-13)


def test_graph_replay_matches_eager():
    """Three steps captured into a HIP graph and replayed several times, with
    eager work and synchronisation between replays: every replay equals the
    eager result of the same number of steps."""
    announce("graph replay")
    torch = need_gpu()
    b = I.config1(grid=(2, 2, 2))
    eager = pb.PatchBatch(b)
    graph = pb.PatchBatch(b)
    for rep in range(3):
        eager.fv_rusanov_step(cfl=0.4, n_steps=3)
        graph.fv_rusanov_step(cfl=0.4, n_steps=3, use_graph=True)
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        np.testing.assert_array_equal(graph.download(), eager.download())
    o, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=9)
    assert np.all(rel_err(b, graph.download(), o) <= 1e-12)
    eager.close()
    graph.close()


@pytest.mark.slow
def test_config1_full_size_parity():
    """The full 2048 x 16^3 Euler batch in the benchmark's launch
    configuration, for the configuration's 20 steps, against the full oracle
    (FP64, then FP32 storage)."""
    announce("config1 full size, 20 steps")
    b = I.config1()
    g, dt, st = run_gpu(b, n_steps=20)
    o, dts, _ = oracle.fv_step(b, cfl=0.4, n_steps=20)
    assert np.all(rel_err(b, g, o) <= 1e-12), rel_err(b, g, o)
    assert abs(dt - dts[-1]) <= 1e-14 * dts[-1]
    # the FP32-storage run of the same workload
    b.state = b.state.astype(np.float32).astype(np.float64)
    announce("config1 full size, 20 steps, fp32 storage")
    g32, _, _ = run_gpu(b, storage="fp32", n_steps=20)
    o32, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=20, round_fp32=True)
    assert np.all(rel_err(b, g32, o32) <= 1e-5), rel_err(b, g32, o32)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_dma_kernel_matches_register_kernel(storage):
    """The DMA-fed 3D kernel (state planes copied HBM -> LDS three planes
    ahead) and the register-prefetch kernel evaluate the same formulas (the
    compiler contracts a few products into FMAs differently, so they agree to
    roundoff, not bitwise), on patches of 4^3, 8^3 and 16^3 (each periodic on
    itself) and several slab depths; both match the oracle."""
    announce(f"dma vs register kernel {storage}")
    ps = np.array([16, 4, 8, 8, 16, 4], np.int32)
    K = len(ps)
    nbr = np.repeat(np.arange(K, dtype=np.int32)[:, None], 6, axis=1)
    cells = int((ps.astype(np.int64) ** 3).sum())
    rho = I.uniform(15, cells, 0.8, 1.2)
    vel = [I.uniform(16 + i, cells, -0.3, 0.3) for i in range(3)]
    pr = I.uniform(19, cells, 0.8, 1.2)
    cons = np.stack(I.euler_prim_to_state(rho, vel, pr, 1.4))
    off = np.concatenate([[0], np.cumsum(ps.astype(np.int64) ** 3)])
    state = np.concatenate([cons[:, off[k]:off[k + 1]].reshape(-1) for k in range(K)])
    if storage == "fp32":
        state = state.astype(np.float32).astype(np.float64)
    b = I.Batch(dim=3, p=ps, dx=1.0 / ps, nbr=nbr, halo=1, pde="euler", params=np.array([1.4]), n_unknowns=5,
                state=state)
    for slab in (0, 3, 8):
        g1, dt1, _ = run_gpu(b, storage=storage, n_steps=4, tuning={"fv_slab": slab, "fv_dma": 1})
        g0, dt0, _ = run_gpu(b, storage=storage, n_steps=4, tuning={"fv_slab": slab, "fv_dma": 0})
        tol = 1e-13 if storage == "fp64" else 1e-6
        assert np.all(rel_err(b, g1, g0) <= tol), rel_err(b, g1, g0)
        assert abs(dt1 - dt0) <= 1e-13 * dt0
        if storage == "fp64":
            o, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=4)
            assert np.all(rel_err(b, g1, o) <= 1e-12)
