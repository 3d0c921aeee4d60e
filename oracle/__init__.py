"""Oracle: plain, slow, double-precision CPU reference of the patch-batch update.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it and shares no code with it.

`oracle.c` (built into liboracle.so next to this file) holds the update
itself: halo fill, CFL step, Rusanov finite volumes, FD4 + Kreiss-Oliger +
RK4, SRHD physics and conservative-to-primitive recovery.  `mlp.py` holds the
multilayer-perceptron reference (forward with the GPU's bfloat16 rounding
points, hand-written backward, Adam) in numpy float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PDE_IDS = {"adv_f": 0, "adv_b": 1, "euler": 2, "linsym": 3, "srhd": 4, "adv_var": 5}


def build(force: bool = True) -> str:
    """Compile oracle.c with strict IEEE flags (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("K", C.c_int), ("N", C.c_int), ("h", C.c_int),
                ("p", C.POINTER(C.c_int)), ("dx", C.POINTER(C.c_double)),
                ("nbr", C.POINTER(C.c_int)), ("pde", C.c_int), ("prm", C.POINTER(C.c_double)),
                ("c2p_tol", C.c_double), ("c2p_maxit", C.c_int), ("M", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("c2p_fail", C.c_long), ("c2p_iters", C.c_long), ("c2p_maxiter_seen", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_fv_step.argtypes = [C.POINTER(_Desc), dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                  dp, C.POINTER(Stats)]
        L.orc_fv_step.restype = C.c_int
        L.orc_fd_step.argtypes = [C.POINTER(_Desc), dp, C.c_double, C.c_double, C.c_double,
                                  C.c_int, C.c_int, dp]
        L.orc_fd_step.restype = C.c_int
        L.orc_cfl_dt.argtypes = [C.POINTER(_Desc), dp, C.c_double, dp]
        L.orc_cfl_dt.restype = C.c_double
        L.orc_halo_blocks.argtypes = [C.POINTER(_Desc), dp, dp]
        L.orc_halo_blocks.restype = C.c_int
        L.orc_con2prim.argtypes = [C.c_long, dp, dp, C.c_double, C.c_double, C.c_int, dp, ip, ip,
                                   C.POINTER(C.c_long)]
        L.orc_con2prim.restype = C.c_long
        L.orc_srhd_prim2cons.argtypes = [C.c_long, dp, dp, C.c_double]
        L.orc_srhd_prim2cons.restype = None
        L.orc_c2p_residual.argtypes = [C.c_double] * 7 + [dp, dp]
        L.orc_c2p_residual.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class _Keep:
    """keeps the numpy arrays behind a descriptor alive"""

    def __init__(self, batch, tol=1e-12, maxit=50):
        self.p = np.ascontiguousarray(batch.p, dtype=np.int32)
        self.dx = np.ascontiguousarray(batch.dx, dtype=np.float64)
        self.nbr = np.ascontiguousarray(batch.nbr, dtype=np.int32).reshape(-1)
        self.prm = np.ascontiguousarray(batch.params, dtype=np.float64)
        if self.prm.size == 0:
            self.prm = np.zeros(1)
        if batch.pde == "srhd" and batch.params.size >= 3:
            tol, maxit = float(batch.params[1]), int(batch.params[2])
        M = batch.dim if batch.pde == "adv_var" else 0   # material parameters: the velocity field
        self.desc = _Desc(batch.dim, batch.K, batch.n_unknowns, batch.halo, _ip(self.p), _dp(self.dx),
                          _ip(self.nbr), PDE_IDS[batch.pde], _dp(self.prm), tol, maxit, M)


class OracleError(RuntimeError):
    pass


def fv_step(batch, state=None, cfl=0.4, dt_fixed=0.0, n_steps=1, round_fp32=False):
    """Rusanov FV steps; returns (new_state, dt_per_step, stats)."""
    q = np.array(batch.state if state is None else state, dtype=np.float64, copy=True)
    k = _Keep(batch)
    dts = np.zeros(max(n_steps, 1))
    st = Stats()
    rc = lib().orc_fv_step(C.byref(k.desc), _dp(q), cfl, dt_fixed, n_steps, int(round_fp32), _dp(dts),
                           C.byref(st))
    if rc:
        raise OracleError(f"orc_fv_step returned {rc}")
    return q, dts[:n_steps], st


def fd_step(batch, state=None, cfl=0.5, dt_fixed=0.0, sigma=0.1, rk_stages=4, n_steps=1):
    q = np.array(batch.state if state is None else state, dtype=np.float64, copy=True)
    k = _Keep(batch)
    dts = np.zeros(max(n_steps, 1))
    rc = lib().orc_fd_step(C.byref(k.desc), _dp(q), cfl, dt_fixed, sigma, rk_stages, n_steps, _dp(dts))
    if rc:
        raise OracleError(f"orc_fd_step returned {rc}")
    return q, dts[:n_steps]


def cfl_dt(batch, state=None, cfl=0.4):
    q = np.ascontiguousarray(batch.state if state is None else state, dtype=np.float64)
    k = _Keep(batch)
    lam = np.zeros(3)
    dt = lib().orc_cfl_dt(C.byref(k.desc), _dp(q), cfl, _dp(lam))
    return dt, lam


def halo_blocks(batch, state=None):
    """list of with-halo AoS blocks [(p+2h)^dim, N] per patch"""
    q = np.ascontiguousarray(batch.state if state is None else state, dtype=np.float64)
    k = _Keep(batch)
    ph = batch.p.astype(np.int64) + 2 * batch.halo
    sizes = ph ** batch.dim * batch.n_unknowns
    out = np.zeros(int(sizes.sum()))
    rc = lib().orc_halo_blocks(C.byref(k.desc), _dp(q), _dp(out))
    if rc:
        raise OracleError(f"orc_halo_blocks returned {rc}")
    res, o = [], 0
    for kk in range(batch.K):
        n = int(sizes[kk])
        shape = (int(ph[kk]),) * batch.dim + (batch.n_unknowns,)
        res.append(out[o:o + n].reshape(shape))
        o += n
    return res


def con2prim(cons, Gam=5.0 / 3.0, tol=1e-12, maxit=50, p_guess=None):
    """cons [5, n] -> (prim [5, n] (rho, vx, vy, vz, p), iters [n], status [n],
    n_fail, n_fallback)"""
    cons = np.ascontiguousarray(cons, dtype=np.float64)
    n = cons.shape[1]
    prim = np.zeros((5, n))
    it = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    nfb = C.c_long(0)
    g = None if p_guess is None else np.ascontiguousarray(p_guess, dtype=np.float64)
    nfail = lib().orc_con2prim(n, _dp(cons), _dp(prim), Gam, tol, maxit,
                               None if g is None else _dp(g), _ip(it), _ip(st), C.byref(nfb))
    return prim, it, st, int(nfail), int(nfb.value)


def srhd_prim2cons(prim, Gam=5.0 / 3.0):
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    out = np.zeros_like(prim)
    lib().orc_srhd_prim2cons(prim.shape[1], _dp(prim), _dp(out), Gam)
    return out


def c2p_residual(cons_cell, Gam, p):
    f = C.c_double()
    df = C.c_double()
    D, Sx, Sy, Sz, tau = (float(v) for v in cons_cell)
    lib().orc_c2p_residual(D, Sx, Sy, Sz, tau, Gam, p, C.byref(f), C.byref(df))
    return f.value, df.value
