"""The measured launch-shape search (pb_autotune): it picks one of its
candidates, leaves the state and the control block untouched, caches its
choice, and the steps that follow still match the oracle."""
import numpy as np
import pytest

import oracle
import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

from gpu_helpers import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu


def check_result(r, n_cand):
    assert not r["from_cache"]
    assert len(r["candidates"]) == n_cand
    us = [t for _, t in r["candidates"]]
    assert all(np.isfinite(t) and t > 0 for t in us)
    assert r["best_us"] == min(us)


def test_fv_autotune_euler3d():
    announce("autotune fv euler3d")
    need_gpu()
    pb.pb_autotune_cache_clear()
    b = I.config1(grid=(4, 4, 2))
    B = pb.PatchBatch(b)
    before, st0 = B.download(), B.stats()
    r = B.autotune("fv", cfl=0.4, trials=2)
    check_result(r, 16)
    plain = [c for c, _ in r["candidates"] if not c["fv_persist"] and not c["fv_column"]]
    assert sorted({c["fv_slab"] for c in plain}) == [4, 8, 16]
    assert {c["fv_column"] for c, _ in r["candidates"]} == {0, 2, 3}
    assert {c["fv_persist"] for c, _ in r["candidates"]} == {0, 3}
    assert {c["fv_dma"] for c, _ in r["candidates"]} == {0, 1}
    assert B.get_tuning() == r["best"]
    np.testing.assert_array_equal(B.download(), before)
    assert B.stats() == st0
    r2 = B.autotune("fv", cfl=0.4, trials=2)
    assert r2["from_cache"] and r2["best"] == r["best"]
    B.fv_rusanov_step(cfl=0.4, n_steps=5)
    g = B.download()
    B.close()
    o, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=5)
    assert np.all(rel_err(b, g, o) <= 1e-12)
    pb.pb_autotune_cache_clear()


def test_fd_autotune_is_bitwise_neutral():
    """FD tunings move tiles between work-groups or split the phases of a tile
    between waves differently: a step after tuning is bitwise equal to a step
    at the default tuning, except with the one-wave-per-tile kernel, which
    adds the K steps of the product in another order (roundoff)."""
    announce("autotune fd")
    need_gpu()
    pb.pb_autotune_cache_clear()
    b = I.config2(n_patches=24, N=20, sizes=np.array([4, 8, 16] * 8, np.int32))
    B = pb.PatchBatch(b)
    before, st0 = B.download(), B.stats()
    r = B.autotune("fd", cfl=0.5, sigma_ko=0.1, trials=2)
    check_result(r, 8)
    assert {c["fd_ws"] for c, _ in r["candidates"]} == {0, 1, 2}
    np.testing.assert_array_equal(B.download(), before)
    assert B.stats() == st0
    B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
    g = B.download()
    B.close()
    B0 = pb.PatchBatch(b)
    B0.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
    g0 = B0.download()
    B0.close()
    if r["best"]["fd_ws"] == 2:
        assert np.all(rel_err(b, g, g0) <= 1e-14)
    else:
        np.testing.assert_array_equal(g, g0)
    o, _ = oracle.fd_step(b, cfl=0.5, sigma=0.1, n_steps=2)
    assert np.all(rel_err(b, g, o) <= 1e-12)
    with pytest.raises(pb.PbError):
        pb.PatchBatch(b).autotune("fv")
    pb.pb_autotune_cache_clear()


def test_euler_fd_autotune():
    """Euler FD: the column-run candidates (2 and 4 work-groups per CU, and
    one work-group per patch) x XCD remap; the state and the statistics are
    untouched, and the steps after tuning equal the default tuning's bits."""
    announce("autotune fd euler")
    need_gpu()
    pb.pb_autotune_cache_clear()
    b = I.config1(grid=(8, 8, 2), p=8, halo=3, seed=12)
    B = pb.PatchBatch(b)
    before, st0 = B.download(), B.stats()
    r = B.autotune("fd", cfl=0.5, sigma_ko=0.1, trials=2)
    check_result(r, 6)
    assert {c["fd_column"] for c, _ in r["candidates"]} == {0, 2, 4}
    assert B.get_tuning() == r["best"]
    np.testing.assert_array_equal(B.download(), before)
    assert B.stats() == st0
    B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
    g = B.download()
    B.close()
    B0 = pb.PatchBatch(b)
    B0.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=2)
    np.testing.assert_array_equal(g, B0.download())
    B0.close()
    # a batch of 4^3 patches runs the small-patch kernel: one candidate
    bs = I.config1(grid=(2, 2, 2), p=4, halo=3, seed=13)
    Bs = pb.PatchBatch(bs)
    rs = Bs.autotune("fd", cfl=0.5, sigma_ko=0.1, trials=2)
    check_result(rs, 1)
    Bs.close()
    pb.pb_autotune_cache_clear()


def test_srhd_autotune_then_step():
    announce("autotune fv srhd")
    need_gpu()
    pb.pb_autotune_cache_clear()
    b = I.config3(grid=(2, 2, 2), seed=31)
    B = pb.PatchBatch(b)
    before, st0 = B.download(), B.stats()
    r = B.autotune("fv", cfl=0.4, trials=2)
    check_result(r, 12)   # SRHD has no DMA-fed kernel: columns (3, 2 per CU), balanced (3) and 3 slabs, x remap
    assert {c["fv_dma"] for c, _ in r["candidates"]} == {0}
    np.testing.assert_array_equal(B.download(), before)
    assert B.stats() == st0
    B.fv_rusanov_step(cfl=0.4, n_steps=2)
    g = B.download()
    B.close()
    o, _, _ = oracle.fv_step(b, cfl=0.4, n_steps=2)
    assert np.all(rel_err(b, g, o) <= 1e-12)
    pb.pb_autotune_cache_clear()
