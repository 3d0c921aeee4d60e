"""MI355X (gfx950) patch-batch library: Python binding of the C ABI declared
in include/patchhip.h.

This module only marshals arguments.  Every step of the update runs in the
HIP kernels of libpatchhip.so; PyTorch provides device memory and the stream.
If the shared library is missing, every entry point raises PbError (there is
no fallback path).

Module-level functions carry the C names (patch_batch_create,
fv_rusanov_step, fd_ko_step, con2prim, pb_mlp_*); `PatchBatch` and `Mlp`
wrap them with torch-owned buffers.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpatchhip.so")

PB_OK, PB_EINVAL, PB_ENOMEM, PB_EHIP, PB_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS = {0: "PB_OK", -1: "PB_EINVAL", -2: "PB_ENOMEM", -3: "PB_EHIP", -4: "PB_EUNSUPPORTED"}
PDE = {"adv_f": 0, "adv_b": 1, "euler": 2, "linsym": 3, "srhd": 4, "adv_var": 5}
STORAGE = {"fp64": 0, "fp32": 1}
GUESS = {"plain": 0, "learned": 1, "warm": 2}
MLP_IN, MLP_HID = 5, 64
MLP_NPARAM = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_HID + 1
MLP_NNORM = 12


class PbError(RuntimeError):
    def __init__(self, what, status, text=""):
        super().__init__(f"{what}: {STATUS.get(status, status)}: {text}")
        self.status = status


class BatchDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_patches", C.c_int32), ("p", C.POINTER(C.c_int32)),
                ("dx", C.POINTER(C.c_double)), ("neighbor", C.POINTER(C.c_int32)), ("halo", C.c_int32),
                ("pde", C.c_int32), ("pde_params", C.POINTER(C.c_double)), ("n_pde_params", C.c_int64),
                ("n_unknowns", C.c_int32), ("n_aux", C.c_int32), ("storage", C.c_int32), ("state", C.c_void_p),
                ("state_alt", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("nonfinite_units", C.c_int64), ("c2p_cells", C.c_int64),
                ("c2p_failures", C.c_int64), ("c2p_iterations", C.c_int64), ("c2p_fallbacks", C.c_int64),
                ("c2p_max_iterations", C.c_int32), ("current", C.c_int32), ("last_dt", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("fv_slab", C.c_int32), ("fv_xcd_remap", C.c_int32), ("fd_xcd_remap", C.c_int32),
                ("fd_wg_per_cu", C.c_int32), ("fv_dma", C.c_int32), ("fd_ws", C.c_int32),
                ("fv_persist", C.c_int32), ("fv_column", C.c_int32), ("fd_column", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PB_TUNE_MAX = 16


class AutotuneResult(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("from_cache", C.c_int32), ("best", C.c_int32),
                ("pad_", C.c_int32), ("cand", Tuning * PB_TUNE_MAX), ("cand_us", C.c_double * PB_TUNE_MAX)]


class OffloadDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("halo", C.c_int32), ("pde", C.c_int32),
                ("pde_params", C.POINTER(C.c_double)), ("n_pde_params", C.c_int64), ("n_unknowns", C.c_int32),
                ("batch_patches", C.c_int32)]


class OffloadTiming(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("pack_ms", C.c_double), ("h2d_ms", C.c_double),
                ("compute_ms", C.c_double), ("d2h_ms", C.c_double), ("unpack_ms", C.c_double),
                ("batches", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded libpatchhip.so (raises PbError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PbError("load", PB_EUNSUPPORTED,
                          f"{LIB_PATH} is not built (python -m paper_2608_19273_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.pb_last_error.restype = C.c_char_p
        L.pb_workspace_size.argtypes = [C.POINTER(BatchDesc), C.POINTER(C.c_size_t)]
        L.patch_batch_create.argtypes = [C.POINTER(BatchDesc), C.POINTER(vp)]
        L.pb_column_runs.argtypes = [C.POINTER(BatchDesc), C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32,
                                     C.POINTER(C.c_int32)]
        L.patch_batch_destroy.argtypes = [vp]
        L.pb_batch_reset.argtypes = [vp, C.c_int32]
        L.pb_batch_stats.argtypes = [vp, C.POINTER(Stats)]
        L.pb_batch_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.pb_batch_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.pb_autotune.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                  C.POINTER(AutotuneResult)]
        L.pb_autotune_cache_save.argtypes = [C.c_char_p]
        L.pb_autotune_cache_load.argtypes = [C.c_char_p, C.POINTER(C.c_int32)]
        L.pb_autotune_cache_clear.argtypes = []
        L.pb_batch_set_c2p_guess.argtypes = [vp, C.c_int32, vp]
        L.pb_batch_profile.argtypes = [vp, C.c_int32]
        L.pb_batch_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.fv_rusanov_step.argtypes = [vp, C.c_double, C.c_double, C.c_int32, C.c_int32, dp]
        L.pb_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.fd_ko_step.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32, dp]
        L.con2prim.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_double, C.c_int32, C.c_int32, vp, vp,
                               vp, vp, vp, vp]
        L.pb_mlp_create.argtypes = [C.POINTER(vp)]
        L.pb_mlp_destroy.argtypes = [vp]
        fp = C.POINTER(C.c_float)
        L.pb_mlp_set_params.argtypes = [vp, fp, fp]
        L.pb_mlp_get_params.argtypes = [vp, fp, fp]
        L.pb_mlp_forward.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.pb_mlp_features.argtypes = [vp, vp, C.c_int64, vp]
        L.pb_mlp_grad.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.pb_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                        C.c_int32, vp, vp]
        L.pb_mlp_prepare.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
        L.pb_mlp_fit_norm.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.pb_mlp_standardise_target.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.pb_mlp_permutation.argtypes = [C.c_uint64, C.c_int64, C.c_int64, vp, vp]
        L.pb_mlp_train_epoch.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_uint64, C.c_int32, C.c_float,
                                         C.c_int64, C.c_int64, C.c_float, C.c_float, C.c_float, vp, vp]
        L.pb_offload_create.argtypes = [C.POINTER(OffloadDesc), C.POINTER(vp)]
        L.pb_offload_destroy.argtypes = [vp]
        L.pb_offload_fv_step.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(vp), dp, C.c_double,
                                         C.POINTER(OffloadTiming)]
        for name in ("pb_offload_create", "pb_offload_destroy", "pb_offload_fv_step"):
            getattr(L, name).restype = C.c_int
        for name in ("pb_workspace_size", "pb_column_runs", "patch_batch_create", "patch_batch_destroy", "pb_batch_reset",
                     "pb_batch_stats", "pb_batch_set_tuning", "pb_batch_get_tuning", "pb_autotune",
                     "pb_autotune_cache_save", "pb_autotune_cache_load", "pb_autotune_cache_clear", "pb_batch_set_c2p_guess", "pb_batch_profile",
                     "pb_batch_profile_read", "pb_stream_copy", "fv_rusanov_step",
                     "fd_ko_step", "con2prim", "pb_mlp_create", "pb_mlp_destroy", "pb_mlp_set_params",
                     "pb_mlp_get_params", "pb_mlp_forward", "pb_mlp_features", "pb_mlp_grad", "pb_mlp_train_step",
                     "pb_mlp_prepare", "pb_mlp_fit_norm", "pb_mlp_standardise_target", "pb_mlp_permutation",
                     "pb_mlp_train_epoch"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pb_last_error().decode()


def _check(rc, what):
    if rc != PB_OK:
        raise PbError(what, rc, last_error())


# ---------------------------------------------------------------- C names --


def pb_workspace_size(desc: BatchDesc) -> int:
    n = C.c_size_t(0)
    _check(lib().pb_workspace_size(C.byref(desc), C.byref(n)), "pb_workspace_size")
    return int(n.value)


def pb_column_runs(desc: BatchDesc, kind: str, w: int, cus: int) -> np.ndarray:
    """the column runs [n, 4] (patch, first plane, planes, 0) that fv_column = w
    (kind "fv") or fd_column = w (kind "fd") sets up on a device of `cus` CUs
    (host-only)"""
    k = {"fv": 0, "fd": 1}[kind]
    n = C.c_int32(0)
    rc = lib().pb_column_runs(C.byref(desc), k, w, cus, None, 0, C.byref(n))
    if rc != PB_OK and n.value == 0:
        _check(rc, "pb_column_runs")
    out = np.zeros((max(n.value, 1), 4), np.int32)
    _check(lib().pb_column_runs(C.byref(desc), k, w, cus, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
           "pb_column_runs")
    return out[:n.value]


def patch_batch_create(desc: BatchDesc):
    h = C.c_void_p()
    _check(lib().patch_batch_create(C.byref(desc), C.byref(h)), "patch_batch_create")
    return h


def patch_batch_destroy(h):
    _check(lib().patch_batch_destroy(h), "patch_batch_destroy")


def fv_rusanov_step(h, cfl=0.4, dt_fixed=0.0, n_steps=1, use_graph=False, want_dt=False):
    dt = C.c_double(0.0)
    _check(lib().fv_rusanov_step(h, cfl, dt_fixed, n_steps, int(use_graph), C.byref(dt) if want_dt else None),
           "fv_rusanov_step")
    return dt.value if want_dt else None


def fd_ko_step(h, cfl=0.5, dt_fixed=0.0, sigma_ko=0.1, rk_stages=4, n_steps=1, use_graph=False, want_dt=False):
    dt = C.c_double(0.0)
    _check(lib().fd_ko_step(h, cfl, dt_fixed, sigma_ko, rk_stages, n_steps, int(use_graph),
                            C.byref(dt) if want_dt else None), "fd_ko_step")
    return dt.value if want_dt else None


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def con2prim(cons, prim, gamma=5.0 / 3.0, tol=1e-12, max_iter=50, guess="plain", mlp=None, p_prev=None,
             iters=None, status=None, counters=None):
    """cons, prim: torch float64 device tensors [5, n]; optional torch outputs."""
    n = cons.shape[-1]
    _check(lib().con2prim(_ptr(cons), _ptr(prim), n, gamma, tol, max_iter, GUESS[guess],
                          None if mlp is None else mlp.handle, _ptr(p_prev), _ptr(iters), _ptr(status),
                          _ptr(counters), _stream()), "con2prim")


def pb_stream_copy(src, dst):
    """device copy src -> dst (torch tensors, same byte size) with the
    library's streaming kernel"""
    n = src.numel() * src.element_size()
    _check(lib().pb_stream_copy(_ptr(src), _ptr(dst), n, _stream()), "pb_stream_copy")


# -------------------------------------------------------------- wrappers --



def pb_autotune(h, kind="fv", cfl=0.4, dt_fixed=0.0, sigma_ko=0.1, trials=5, use_cache=True):
    r = AutotuneResult()
    k = {"fv": 0, "fd": 1}[kind] if isinstance(kind, str) else int(kind)
    _check(lib().pb_autotune(h, k, cfl, dt_fixed, sigma_ko, int(trials), int(bool(use_cache)), C.byref(r)),
           "pb_autotune")
    cands = [(r.cand[i].as_dict(), r.cand_us[i]) for i in range(r.n_candidates)]
    return {"best": cands[r.best][0], "best_us": cands[r.best][1], "from_cache": bool(r.from_cache),
            "candidates": cands}


def pb_autotune_cache_save(path):
    _check(lib().pb_autotune_cache_save(os.fsencode(path)), "pb_autotune_cache_save")


def pb_autotune_cache_load(path) -> int:
    n = C.c_int32(0)
    _check(lib().pb_autotune_cache_load(os.fsencode(path), C.byref(n)), "pb_autotune_cache_load")
    return n.value


def pb_autotune_cache_clear():
    _check(lib().pb_autotune_cache_clear(), "pb_autotune_cache_clear")


class Mlp:
    """The learned con2prim guess network (library-owned device parameters)."""

    def __init__(self, params=None, norm=None):
        h = C.c_void_p()
        _check(lib().pb_mlp_create(C.byref(h)), "pb_mlp_create")
        self.handle = h
        if params is not None:
            self.set_params(params, norm)

    def close(self):
        if self.handle:
            lib().pb_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, norm):
        p = np.ascontiguousarray(params, dtype=np.float32)
        nn = np.ascontiguousarray(norm, dtype=np.float32)
        assert p.size == MLP_NPARAM and nn.size == MLP_NNORM
        fp = C.POINTER(C.c_float)
        _check(lib().pb_mlp_set_params(self.handle, p.ctypes.data_as(fp), nn.ctypes.data_as(fp)),
               "pb_mlp_set_params")

    def get_params(self):
        p = np.zeros(MLP_NPARAM, np.float32)
        nn = np.zeros(MLP_NNORM, np.float32)
        fp = C.POINTER(C.c_float)
        _check(lib().pb_mlp_get_params(self.handle, p.ctypes.data_as(fp), nn.ctypes.data_as(fp)),
               "pb_mlp_get_params")
        return p, nn

    def forward(self, x):
        """x: torch float32 device [n, 5] raw features -> torch [n]"""
        import torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(lib().pb_mlp_forward(self.handle, _ptr(x), _ptr(y), x.shape[0], _stream()), "pb_mlp_forward")
        return y

    def grad(self, x, t):
        import torch
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().pb_mlp_grad(self.handle, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _stream()),
               "pb_mlp_grad")
        return g, loss

    def train_step(self, x, t, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, loss=None):
        _check(lib().pb_mlp_train_step(self.handle, _ptr(x), _ptr(t), x.shape[0], lr, beta1, beta2, eps, step,
                                       _ptr(loss), _stream()), "pb_mlp_train_step")

    def fit_norm(self, x, y):
        """normalisation statistics of the training set (device) -> this
        network's normalisation block"""
        _check(lib().pb_mlp_fit_norm(self.handle, _ptr(x), _ptr(y), x.shape[0], _stream()), "pb_mlp_fit_norm")

    def standardise_target(self, y):
        """t = (y - y_mean) / y_std with this network's statistics (device)"""
        import torch
        t = torch.empty_like(y)
        _check(lib().pb_mlp_standardise_target(self.handle, _ptr(y), _ptr(t), y.shape[0], _stream()),
               "pb_mlp_standardise_target")
        return t

    def train_epoch(self, x, t, batch, seed, epoch, lr_max, step0, total_steps, loss_sum=None, beta1=0.9,
                    beta2=0.999, eps=1e-8):
        """one epoch of Adam steps over batches of the seeded permutation of
        the rows (cosine learning rate over total_steps); loss_sum (device
        float64 [1], nullable) accumulates the batch losses"""
        _check(lib().pb_mlp_train_epoch(self.handle, _ptr(x), _ptr(t), x.shape[0], batch, seed, epoch, lr_max, step0,
                                        total_steps, beta1, beta2, eps, _ptr(loss_sum), _stream()),
               "pb_mlp_train_epoch")


def pb_mlp_prepare(cons, p):
    """training inputs of conserved states cons [5, n] (float64 device) and
    their pressures p [n]: raw features [n, 5] and targets log(p/E) [n]
    (float32 device)"""
    import torch
    n = cons.shape[-1]
    x = torch.empty((n, MLP_IN), dtype=torch.float32, device=cons.device)
    y = torch.empty(n, dtype=torch.float32, device=cons.device)
    _check(lib().pb_mlp_prepare(_ptr(cons), _ptr(p), _ptr(x), _ptr(y), n, _stream()), "pb_mlp_prepare")
    return x, y


def pb_mlp_permutation(seed, epoch, n, device="cuda"):
    """the library's seeded permutation of [0, n) for (seed, epoch) (int64 device)"""
    import torch
    idx = torch.empty(n, dtype=torch.int64, device=device)
    _check(lib().pb_mlp_permutation(seed, epoch, n, _ptr(idx), _stream()), "pb_mlp_permutation")
    return idx


def pb_mlp_features(cons):
    """cons: torch float64 device [5, n] -> raw features torch float32 [n, 5]"""
    import torch
    n = cons.shape[-1]
    x = torch.empty((n, MLP_IN), dtype=torch.float32, device=cons.device)
    _check(lib().pb_mlp_features(_ptr(cons), _ptr(x), n, _stream()), "pb_mlp_features")
    return x


class PatchBatch:
    """A patch batch whose state lives in two torch device buffers."""

    def __init__(self, batch, storage="fp64", device="cuda", state=None):
        import torch
        self.batch = batch
        self.storage = storage
        self.dtype = torch.float64 if storage == "fp64" else torch.float32
        self.device = torch.device(device)
        n = batch.total_cells * batch.n_unknowns
        self.bufs = [torch.empty(n, dtype=self.dtype, device=self.device),
                     torch.empty(n, dtype=self.dtype, device=self.device)]
        src = batch.state if state is None else state
        self.bufs[0].copy_(torch.from_numpy(np.ascontiguousarray(src)).to(self.dtype))
        self._p = np.ascontiguousarray(batch.p, dtype=np.int32)
        self._dx = np.ascontiguousarray(batch.dx, dtype=np.float64)
        self._nbr = np.ascontiguousarray(batch.nbr, dtype=np.int32).reshape(-1)
        self._prm = np.ascontiguousarray(batch.params, dtype=np.float64)
        self.desc = BatchDesc(batch.dim, batch.K, self._p.ctypes.data_as(C.POINTER(C.c_int32)),
                              self._dx.ctypes.data_as(C.POINTER(C.c_double)),
                              self._nbr.ctypes.data_as(C.POINTER(C.c_int32)), batch.halo, PDE[batch.pde],
                              self._prm.ctypes.data_as(C.POINTER(C.c_double)), self._prm.size,
                              batch.n_unknowns - batch.n_aux, batch.n_aux, STORAGE[storage], self.bufs[0].data_ptr(),
                              self.bufs[1].data_ptr(), None, 0, _stream())
        ws = pb_workspace_size(self.desc)
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.desc.workspace = aligned
        self.desc.workspace_bytes = ws
        self.handle = patch_batch_create(self.desc)

    def close(self):
        if self.handle:
            patch_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fv_rusanov_step(self, cfl=0.4, dt_fixed=0.0, n_steps=1, use_graph=False, want_dt=False):
        return fv_rusanov_step(self.handle, cfl, dt_fixed, n_steps, use_graph, want_dt)

    def fd_ko_step(self, cfl=0.5, dt_fixed=0.0, sigma_ko=0.1, rk_stages=4, n_steps=1, use_graph=False,
                   want_dt=False):
        return fd_ko_step(self.handle, cfl, dt_fixed, sigma_ko, rk_stages, n_steps, use_graph, want_dt)

    def stats(self) -> dict:
        s = Stats()
        _check(lib().pb_batch_stats(self.handle, C.byref(s)), "pb_batch_stats")
        return s.as_dict()

    def current(self):
        return self.bufs[self.stats()["current"]]

    def download(self) -> np.ndarray:
        return self.current().double().cpu().numpy()

    def reset(self, state=None):
        import torch
        if state is not None:
            self.bufs[0].copy_(torch.from_numpy(np.ascontiguousarray(state)).to(self.dtype))
        _check(lib().pb_batch_reset(self.handle, 0), "pb_batch_reset")

    def set_tuning(self, fv_slab=0, fv_xcd_remap=1, fd_xcd_remap=1, fd_wg_per_cu=2, fv_dma=0, fd_ws=1,
                   fv_persist=0, fv_column=0, fd_column=2):
        t = Tuning(fv_slab, fv_xcd_remap, fd_xcd_remap, fd_wg_per_cu, fv_dma, fd_ws, fv_persist, fv_column, fd_column)
        _check(lib().pb_batch_set_tuning(self.handle, C.byref(t)), "pb_batch_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(lib().pb_batch_get_tuning(self.handle, C.byref(t)), "pb_batch_get_tuning")
        return t.as_dict()

    def autotune(self, kind="fv", cfl=0.4, dt_fixed=0.0, sigma_ko=0.1, trials=5, use_cache=True):
        """measured launch-shape search (pb_autotune); returns the chosen tuning
        and the measured candidates"""
        return pb_autotune(self.handle, kind, cfl, dt_fixed, sigma_ko, trials, use_cache)

    def profile(self, on=True, span=False):
        """on: time each step kernel launch with an event pair; span: one pair
        over the back-to-back step launches of an FV call (not SRHD)"""
        _check(lib().pb_batch_profile(self.handle, (2 if span else 1) if on else 0), "pb_batch_profile")

    def profile_read(self):
        """(total ms, launches) of the step kernels recorded since the last read
        (in span mode the ms are the span of the launches they cover)"""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        _check(lib().pb_batch_profile_read(self.handle, C.byref(ms), C.byref(n)), "pb_batch_profile_read")
        return ms.value, n.value

    def set_c2p_guess(self, guess="plain", mlp=None):
        _check(lib().pb_batch_set_c2p_guess(self.handle, GUESS[guess], None if mlp is None else mlp.handle),
               "pb_batch_set_c2p_guess")


class Offload:
    """Offload mode (pb_offload_*): K patches handed over as K host arrays,
    each the (p+2h)^3 halo box in per-point order [z][y][x][N], returned as K
    host arrays [p][p][p][N] of updated interiors."""

    def __init__(self, p, halo, pde, params, n_unknowns, batch_patches=0):
        self._prm = np.ascontiguousarray(params, dtype=np.float64)
        d = OffloadDesc(3, p, halo, PDE[pde], self._prm.ctypes.data_as(C.POINTER(C.c_double)), self._prm.size,
                        n_unknowns, batch_patches)
        h = C.c_void_p()
        _check(lib().pb_offload_create(C.byref(d), C.byref(h)), "pb_offload_create")
        self.handle = h
        self.p, self.halo, self.N = p, halo, n_unknowns

    def fv_step(self, chunks_in, chunks_out, dx, dt) -> dict:
        """chunks_in / chunks_out: lists of C-contiguous float64 numpy arrays
        ((p+2h)^3 * N and p^3 * N values); dx: K cell widths"""
        K = len(chunks_in)
        if len(chunks_out) != K:
            raise ValueError("chunks_in and chunks_out differ in length")
        for a in list(chunks_in) + list(chunks_out):
            if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
                raise ValueError("chunks must be C-contiguous float64 arrays")
        ins = (C.c_void_p * max(K, 1))(*[a.ctypes.data for a in chunks_in])
        outs = (C.c_void_p * max(K, 1))(*[a.ctypes.data for a in chunks_out])
        dxa = np.ascontiguousarray(dx, dtype=np.float64)
        t = OffloadTiming()
        _check(lib().pb_offload_fv_step(self.handle, K, ins, outs, dxa.ctypes.data_as(C.POINTER(C.c_double)),
                                        dt, C.byref(t)), "pb_offload_fv_step")
        return t.as_dict()

    def close(self):
        if self.handle is not None:
            _check(lib().pb_offload_destroy(self.handle), "pb_offload_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
