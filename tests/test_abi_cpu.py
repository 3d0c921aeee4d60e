"""The C-ABI library loads, exports every entry point include/patchhip.h
declares, and rejects bad arguments on the host before any HIP call (these
tests run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "patchhip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert {"patch_batch_create", "fv_rusanov_step", "fd_ko_step", "con2prim"} <= set(names)
    L = pb.lib()
    for n in names:
        assert hasattr(L, n), n


def desc_for(b, state=1, alt=2, ws=256, ws_bytes=1 << 40, storage=0, **over):
    p = np.ascontiguousarray(b.p, np.int32)
    dx = np.ascontiguousarray(b.dx, np.float64)
    nbr = np.ascontiguousarray(b.nbr, np.int32).reshape(-1)
    prm = np.ascontiguousarray(b.params, np.float64)
    keep = (p, dx, nbr, prm)
    d = pb.BatchDesc(b.dim, b.K, p.ctypes.data_as(C.POINTER(C.c_int32)), dx.ctypes.data_as(C.POINTER(C.c_double)),
                     nbr.ctypes.data_as(C.POINTER(C.c_int32)), b.halo, pb.PDE[b.pde],
                     prm.ctypes.data_as(C.POINTER(C.c_double)), prm.size, b.n_unknowns - b.n_aux, b.n_aux, storage,
                     state, alt, ws, ws_bytes, None)
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


def test_workspace_size_layout():
    def a256(v):
        return (v + 255) // 256 * 256

    def part(K):  # per-unit partials [8][16 K] doubles + second-stage [8][16 K / 256 + 1]
        return a256(8 * (16 * K + 16 * K // 256 + 1) * 8)

    b = I.config0()
    d, keep = desc_for(b)
    assert pb.pb_workspace_size(d) == 256 + part(b.K)
    b3 = I.config3(grid=(2, 2, 1), p=4)
    d, keep = desc_for(b3)
    assert pb.pb_workspace_size(d) == 256 + part(b3.K) + a256(b3.total_cells * 8)
    b2 = I.config2(n_patches=8, N=58, sizes=np.array([4] * 8, np.int32))
    d, keep = desc_for(b2)
    per = a256(b2.total_cells * 58 * 8)
    assert pb.pb_workspace_size(d) == 256 + part(b2.K) + 2 * per


def test_material_parameter_counts():
    """n_aux (M material parameters per point): the variable-advection
    batch takes n_unknowns = 1 and n_aux = dim; M > 0 for another PDE is a
    valid request the library does not implement; either is reported before
    any HIP call"""
    b = I.adv_var_batch((2, 2, 1), 4)
    d, keep = desc_for(b)
    assert (d.n_unknowns, d.n_aux) == (1, 3)
    assert pb.pb_workspace_size(d) > 0
    h = C.c_void_p()
    for n, m, rc, msg in ((4, 0, pb.PB_EINVAL, "n_aux = dim"), (1, 2, pb.PB_EINVAL, "n_aux = dim"),
                          (1, -1, pb.PB_EINVAL, "n_aux")):
        d.n_unknowns, d.n_aux = n, m
        assert pb.lib().patch_batch_create(C.byref(d), C.byref(h)) == rc
        assert msg in pb.last_error() and not h.value
    e, keep2 = desc_for(I.config0())
    e.n_aux = 1
    assert pb.lib().patch_batch_create(C.byref(e), C.byref(h)) == pb.PB_EUNSUPPORTED
    assert "ADVECTION_VAR" in pb.last_error() and not h.value


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 4, "dim"), ("n_patches", 0, "n_patches"), ("halo", 0, "halo"), ("pde", 9, "pde"),
    ("n_unknowns", 3, "n_unknowns"), ("storage", 7, "storage"), ("n_pde_params", 0, "pde_params"),
    ("state", None, "state"), ("workspace", None, "workspace"), ("workspace", 128, "aligned"),
    ("workspace_bytes", 16, "too small"),
])
def test_create_rejects_bad_descriptors_without_gpu(field, value, msg):
    b = I.config0()
    d, keep = desc_for(b)
    setattr(d, field, value)
    h = C.c_void_p()
    rc = pb.lib().patch_batch_create(C.byref(d), C.byref(h))
    assert rc == pb.PB_EINVAL
    assert msg in pb.last_error()
    assert not h.value


def test_create_rejects_bad_tables():
    b = I.config0()
    b.nbr = b.nbr.copy()
    b.nbr[3, 1] = 999
    d, keep = desc_for(b)
    assert pb.lib().patch_batch_create(C.byref(d), C.byref(C.c_void_p())) == pb.PB_EINVAL
    assert "neighbour" in pb.last_error()
    b = I.config0()
    b.dx = b.dx.copy()
    b.dx[2] = -1.0
    d, keep = desc_for(b)
    assert pb.lib().patch_batch_create(C.byref(d), C.byref(C.c_void_p())) == pb.PB_EINVAL
    b = I.make_uniform_batch((2, 2), 2, 3, "euler", [1.4], 4, 0.1)  # p < halo
    d, keep = desc_for(b)
    assert pb.lib().patch_batch_create(C.byref(d), C.byref(C.c_void_p())) == pb.PB_EINVAL
    assert "halo" in pb.last_error()
    b = I.config3(grid=(2, 1, 1), p=4)
    b.params = np.array([5 / 3, 0.0, 50])  # tol 0
    d, keep = desc_for(b)
    assert pb.lib().patch_batch_create(C.byref(d), C.byref(C.c_void_p())) == pb.PB_EINVAL


def test_null_handles_rejected():
    L = pb.lib()
    assert L.fv_rusanov_step(None, 0.4, 0.0, 1, 0, None) == pb.PB_EINVAL
    assert L.fd_ko_step(None, 0.5, 0.0, 0.1, 4, 1, 0, None) == pb.PB_EINVAL
    assert L.pb_batch_stats(None, None) == pb.PB_EINVAL
    assert L.pb_workspace_size(None, None) == pb.PB_EINVAL
    assert L.patch_batch_destroy(None) == pb.PB_OK


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pb, "_lib", None)
    with pytest.raises(pb.PbError):
        pb.lib()


def test_autotune_rejects_bad_arguments_without_gpu():
    L = pb.lib()
    r = pb.AutotuneResult()
    assert L.pb_autotune(None, 0, 0.4, 0.0, 0.1, 5, 1, C.byref(r)) == pb.PB_EINVAL
    assert L.pb_batch_get_tuning(None, None) == pb.PB_EINVAL
    assert L.pb_batch_set_tuning(None, None) == pb.PB_EINVAL


def test_autotune_cache_file_round_trip(tmp_path):
    """the tuning cache is host-side: entries load, save and reload unchanged
    (lines of six, seven or eight fields load the missing ones at their
    defaults: fv_persist 0, fv_column 0, fd_column 2); a malformed line is
    rejected with the entries before it kept"""
    pb.pb_autotune_cache_clear()
    src = tmp_path / "in.txt"
    src.write_text("fv/pde2/d3/N5/s0/h1/16x2048 8 1 1 2 1 1 1\n\nfd/pde3/d3/N58/s0/h3/4x1024,8x2048,16x1024 0 1 0 1 0 0\n"
                   "fv/pde2/d3/N5/s0/h1/16x768 0 1 1 2 0 1 0 3\nfd/pde2/d3/N5/s0/h3/16x2048 0 1 1 2 0 1 0 0 4\n")
    assert pb.pb_autotune_cache_load(str(src)) == 4
    out = tmp_path / "out.txt"
    pb.pb_autotune_cache_save(str(out))
    lines = sorted(out.read_text().splitlines())
    assert lines == sorted(["fv/pde2/d3/N5/s0/h1/16x2048 8 1 1 2 1 1 1 0 2",
                            "fd/pde3/d3/N58/s0/h3/4x1024,8x2048,16x1024 0 1 0 1 0 0 0 0 2",
                            "fv/pde2/d3/N5/s0/h1/16x768 0 1 1 2 0 1 0 3 2",
                            "fd/pde2/d3/N5/s0/h3/16x2048 0 1 1 2 0 1 0 0 4"])
    bad = tmp_path / "bad.txt"
    bad.write_text("fv/x 4 1 1 2 1 1\nfv/y 99 1 1 2 1 1\nfv/z 4 1 1 2 1 1\n")
    with pytest.raises(pb.PbError, match="bad2.txt:1"):
        bad2 = tmp_path / "bad2.txt"
        bad2.write_text("fv/w 4 1 1 2 1 1 9\n")
        pb.pb_autotune_cache_load(str(bad2))
    with pytest.raises(pb.PbError, match="bad3.txt:1"):
        bad3 = tmp_path / "bad3.txt"
        bad3.write_text("fv/v 4 1 1 2 1 1 0 9\n")
        pb.pb_autotune_cache_load(str(bad3))
    with pytest.raises(pb.PbError, match="bad4.txt:1"):
        bad4 = tmp_path / "bad4.txt"
        bad4.write_text("fv/u 4 1 1 2 1 1 0 3 9\n")
        pb.pb_autotune_cache_load(str(bad4))
    with pytest.raises(pb.PbError, match="bad5.txt:1"):
        bad5 = tmp_path / "bad5.txt"
        bad5.write_text("fv/t 4 1 1 2 1 1 0 3 2 1\n")
        pb.pb_autotune_cache_load(str(bad5))
    with pytest.raises(pb.PbError, match="bad.txt:2"):
        pb.pb_autotune_cache_load(str(bad))
    pb.pb_autotune_cache_save(str(out))
    keys = {ln.split()[0] for ln in out.read_text().splitlines()}
    assert "fv/x" in keys and "fv/y" not in keys and "fv/z" not in keys
    with pytest.raises(pb.PbError):
        pb.pb_autotune_cache_load(str(tmp_path / "missing.txt"))
    pb.pb_autotune_cache_clear()
    pb.pb_autotune_cache_save(str(out))
    assert out.read_text() == ""


def test_offload_create_rejects_bad_descriptions():
    """pb_offload_create checks its description before allocating anything."""
    L = pb.lib()
    prm = np.array([1.4, 0.0, 0.0, 0.0])

    def create(**kw):
        f = dict(dim=3, p=8, halo=1, pde=pb.PDE["euler"], n_unknowns=5, batch_patches=0, n=1)
        f.update(kw)
        d = pb.OffloadDesc(f["dim"], f["p"], f["halo"], f["pde"], prm.ctypes.data_as(C.POINTER(C.c_double)),
                           f["n"], f["n_unknowns"], f["batch_patches"])
        h = C.c_void_p()
        return L.pb_offload_create(C.byref(d), C.byref(h))

    assert create(dim=2) == pb.PB_EUNSUPPORTED
    assert create(p=0) == pb.PB_EINVAL
    assert create(p=17) == pb.PB_EINVAL
    assert create(halo=0) == pb.PB_EINVAL
    assert create(pde=pb.PDE["linsym"]) == pb.PB_EUNSUPPORTED
    assert create(pde=pb.PDE["srhd"]) == pb.PB_EUNSUPPORTED
    assert create(n_unknowns=4) == pb.PB_EINVAL
    assert create(n=0) == pb.PB_EINVAL
    assert create(batch_patches=-1) == pb.PB_EINVAL
    assert L.pb_offload_fv_step(None, 1, None, None, None, 1e-3, None) == pb.PB_EINVAL
    assert L.pb_offload_destroy(None) == pb.PB_EINVAL


def _check_runs(b, runs, w, cus, pmin=2):
    """every plane of every patch in exactly one run; inside a run the plane
    after a patch top is the +z neighbour's first plane, and only along a link
    (the neighbour's -z neighbour is the patch, same p >= pmin)"""
    count = [np.zeros(int(pk), np.int32) for pk in b.p]
    for k, z0, n, pad in runs:
        assert pad == 0 and n >= 1 and 0 <= z0 < b.p[k]
        z = z0
        for _ in range(n):
            count[k][z] += 1
            z += 1
            if z == b.p[k]:
                s = b.nbr[k, 5]
                k_next, z = s, 0
                if _ + 1 < n:   # the run continues: only along a link
                    assert b.nbr[s, 4] == k and b.p[s] == b.p[k] >= pmin
                k = k_next
    for c in count:
        np.testing.assert_array_equal(c, 1)
    planes = int(b.p.astype(np.int64).sum())
    assert len(runs) <= planes


@pytest.mark.parametrize("grid,w", [((16, 16, 8), 3), ((8, 8, 3), 1), ((8, 8, 3), 3), ((4, 4, 2), 2),
                                    ((16, 16, 3), 2)])
def test_column_runs_cover_every_plane(grid, w):
    """The column-run schedule (pb_column_runs, the table fv_column = w
    uploads): z-periodic grids give one cycle per column; the runs of a
    column split its planes evenly and, with enough planes, number about
    w * 256 in total; the table is layer-major: the lowest run of every
    chain (chains in order of their smallest patch), then the second, ..."""
    b = I.make_uniform_batch(grid, 16, 1, "euler", [1.4], 5, 1.0 / 16)
    d, keep = desc_for(b)
    runs = pb.pb_column_runs(d, "fv", w, 256)
    _check_runs(b, runs, w, 256)
    nx, ny, nz = grid
    columns = nx * ny
    planes_per_col = nz * 16
    per_col = max(1, min(planes_per_col, round(w * 256 * planes_per_col / (columns * planes_per_col))))
    assert len(runs) == columns * per_col
    # run j of column c (patches c, c + nx ny, ...) is unit j columns + c; a column's runs split it evenly
    for c in range(columns):
        rc = runs[c::columns]
        starts = [(k // columns) * 16 + z0 for k, z0, n, _ in rc]
        assert all(k % columns == c for k, _, _, _ in rc)
        assert starts == [j * planes_per_col // per_col for j in range(per_col)]


def test_column_runs_open_chains_and_ragged():
    """Open z chains (bottom and top patches are their own outer z
    neighbours), a ragged batch whose patches are their own z neighbours, and
    the query's error paths."""
    b = I.make_uniform_batch((4, 4, 3), 8, 1, "euler", [1.4], 5, 1.0 / 8)
    layer = 16
    for k in range(b.K):
        if k // layer == 0:
            b.nbr[k, 4] = k
        if k // layer == 2:
            b.nbr[k, 5] = k
    d, keep = desc_for(b)
    for w in (1, 3, 8):
        runs = pb.pb_column_runs(d, "fv", w, 4)
        _check_runs(b, runs, w, 4)
        # 16 chains of 24 planes, 4 w slots: runs per chain round(w / 4), at least 1
        assert len(runs) == 16 * max(1, round(w * 4 / 16))
    # a chain of one patch per patch when the +z neighbour is itself
    ps = np.array([5, 5, 11, 16, 11], np.int32)
    nbr = np.array([[1, 1, 0, 0, 0, 0], [0, 0, 1, 1, 1, 1], [4, 4, 2, 2, 2, 2], [3] * 6, [2, 2, 4, 4, 4, 4]],
                   np.int32)
    rb = I.Batch(dim=3, p=ps, dx=1.0 / ps, nbr=nbr, halo=1, pde="euler", params=np.array([1.4]), n_unknowns=5,
                 state=np.zeros(5 * int((ps.astype(np.int64) ** 3).sum())))
    d2, keep2 = desc_for(rb)
    runs = pb.pb_column_runs(d2, "fv", 3, 256)
    _check_runs(rb, runs, 3, 256)
    assert len(runs) == int(ps.sum())   # more slots than planes: one run per plane
    n = C.c_int32(-1)
    assert pb.lib().pb_column_runs(C.byref(d2), 0, 3, 256, None, 0, C.byref(n)) == pb.PB_EINVAL
    assert n.value == len(runs)
    assert pb.lib().pb_column_runs(C.byref(d2), 0, 0, 256, None, 0, C.byref(n)) == pb.PB_EINVAL
    assert pb.lib().pb_column_runs(C.byref(d2), 0, 9, 256, None, 0, C.byref(n)) == pb.PB_EINVAL
    b2 = I.config0()
    d3, keep3 = desc_for(b2)
    assert pb.lib().pb_column_runs(C.byref(d3), 0, 3, 256, None, 0, C.byref(n)) == pb.PB_EINVAL
    assert pb.lib().pb_column_runs(C.byref(d2), 2, 3, 256, None, 0, C.byref(n)) == pb.PB_EINVAL


@pytest.mark.parametrize("grid,w,per_col", [((16, 16, 8), 2, 2), ((16, 16, 8), 4, 4), ((8, 8, 3), 2, 3),
                                            ((4, 4, 2), 8, 2)])
def test_fd_column_runs_whole_patches(grid, w, per_col):
    """The Euler FD rule (fd_column): runs are whole patches at least, so a
    column of nz patches gets at most nz runs, and the halo of 3 needs
    p >= 4 for a link: a batch of 3^3 patches has no links (one run per
    patch)."""
    b = I.make_uniform_batch(grid, 16, 3, "euler", [1.4], 5, 1.0 / 16)
    d, keep = desc_for(b)
    runs = pb.pb_column_runs(d, "fd", w, 256)
    _check_runs(b, runs, w, 256, pmin=4)
    nx, ny, nz = grid
    assert len(runs) == nx * ny * per_col
    assert np.all(runs[:, 2] >= 16)
    b3 = I.make_uniform_batch((4, 4, 4), 3, 3, "euler", [1.4], 5, 1.0 / 3)
    d3, keep3 = desc_for(b3)
    runs3 = pb.pb_column_runs(d3, "fd", 2, 256)
    _check_runs(b3, runs3, 2, 256, pmin=4)
    assert len(runs3) == b3.K and np.all(runs3[:, 1] == 0) and np.all(runs3[:, 2] == 3)
    # the FV rule links p = 3 patches (one chain per column of 4) and splits finer
    runs3v = pb.pb_column_runs(d3, "fv", 2, 256)
    _check_runs(b3, runs3v, 2, 256)
    assert len(runs3v) > b3.K
