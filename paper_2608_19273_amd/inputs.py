"""Seeded synthetic inputs for the patch-batch update.

This module only *builds inputs*: patch tables (sizes, cell widths, face
neighbours), initial states and physics parameters.  It holds none of the
update's arithmetic (no flux, no eigenvalue, no time step, no
conservative-to-primitive recovery); the HIP library and the oracle both
receive exactly the arrays made here.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), evaluated as a counter-based
generator: output i of a stream with seed s is mix(s + (i+1)*0x9E3779B97F4A7C15).
Uniform doubles take the top 53 bits.  Normal variates use Box-Muller.

State layout ("exchange layout", patch-blocked structure of arrays): patch k
with p_k cells per direction owns the contiguous range
[off_k*N, (off_k + p_k^d)*N); inside it unknown v occupies p_k^d consecutive
values with the cell index (z*p + y)*p + x, x fastest.

Workload recipes (the paper's workloads are not public data sets; every input
here is synthetic and seeded):
  c0  2D Euler (gamma 1.4), 64x64 periodic cells on [0,1]^2 as 8x8 patches of
      8^2 cells, density 1 + 0.2 sin(2 pi x) sin(2 pi y), velocity (0.5, 0.3),
      pressure 1, sampled at cell centres.
  c1  3D Euler, 2048 patches of 16^3 arranged 16x16x8 (x fastest), 256x256x128
      cells, dx = 1/256 on [0,1]x[0,1]x[0,1/2], periodic; each primitive is a
      normalised sum of 8 random Fourier modes, density and pressure in
      [0.5, 1.5], |v| < 0.5.
  c2  linear symmetric system with 58 unknowns, 4096 independent periodic
      unit-cube patches of 4^3, 8^3, 16^3 in exact ratio 1:2:1 in shuffled
      order, per (patch, unknown) four Fourier modes of amplitude in
      [-1/4, 1/4]; B_d = A_d / rho(A_d) with A_d the symmetric part of a
      Gaussian matrix.
  c3  3D special-relativistic hydrodynamics (Gamma 5/3), same grid as c1,
      primitives i.i.d. per cell: rho, eps log-uniform in [1e-3, 10],
      Lorentz factor uniform in [1, 10], isotropic velocity direction.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+n-1 of the SplitMix64 sequence seeded with `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN)


def substream(seed: int, *keys: int) -> int:
    """A derived seed for an independent stream (hash of seed and keys)."""
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for k in keys:
            s = _mix(np.array([s ^ (np.uint64(k & 0xFFFFFFFFFFFFFFFF) * _M2)], dtype=np.uint64))[0]
    return int(s)


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def normal(seed: int, n: int) -> np.ndarray:
    """Box-Muller on pairs of uniforms (the first uniform mapped into (0,1])."""
    m = (n + 1) // 2
    u = uniform(seed, 2 * m)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)])
    return z[:n]


# ----------------------------------------------------------------- batch --


@dataclasses.dataclass
class Batch:
    """A patch batch description plus its state in the exchange layout."""

    dim: int
    p: np.ndarray          # int32 [K]
    dx: np.ndarray         # float64 [K]
    nbr: np.ndarray        # int32 [K, 2*dim]  (-x,+x,-y,+y,-z,+z)
    halo: int
    pde: str               # 'adv_f' | 'adv_b' | 'euler' | 'linsym' | 'srhd'
    params: np.ndarray     # float64, meaning depends on pde
    n_unknowns: int
    state: np.ndarray      # float64 [total_cells * N], exchange layout
    origin: np.ndarray | None = None  # float64 [K, dim] lower corner of each patch

    @property
    def K(self) -> int:
        return int(self.p.shape[0])

    @property
    def n_aux(self) -> int:
        """material parameters among the n_unknowns values per point (the
        velocity field of variable advection)"""
        return self.dim if self.pde == "adv_var" else 0

    def cells(self) -> np.ndarray:
        return self.p.astype(np.int64) ** self.dim

    def offsets(self) -> np.ndarray:
        c = self.cells()
        off = np.zeros(self.K + 1, dtype=np.int64)
        np.cumsum(c, out=off[1:])
        return off

    @property
    def total_cells(self) -> int:
        return int(self.cells().sum())

    def copy(self) -> "Batch":
        return dataclasses.replace(self, state=self.state.copy())

    def patch_view(self, state: np.ndarray, k: int) -> np.ndarray:
        """[N, p, p(, p)] view (z, y, x order) of patch k in `state`."""
        off = self.offsets()
        p = int(self.p[k])
        shape = (self.n_unknowns,) + (p,) * self.dim
        return state[off[k] * self.n_unknowns:(off[k] + p ** self.dim) * self.n_unknowns].reshape(shape)

    def to_global(self, state: np.ndarray, grid: tuple[int, ...]) -> np.ndarray:
        """Uniform-p batch on a patch grid (nx, ny[, nz], x fastest) -> global
        array [N, (Z,) Y, X]."""
        p = int(self.p[0])
        N = self.n_unknowns
        if self.dim == 2:
            nx, ny = grid
            a = state.reshape(ny, nx, N, p, p)
            return a.transpose(2, 0, 3, 1, 4).reshape(N, ny * p, nx * p)
        nx, ny, nz = grid
        a = state.reshape(nz, ny, nx, N, p, p, p)
        return a.transpose(3, 0, 4, 1, 5, 2, 6).reshape(N, nz * p, ny * p, nx * p)

    def from_global(self, g: np.ndarray, grid: tuple[int, ...]) -> np.ndarray:
        p = int(self.p[0])
        N = self.n_unknowns
        if self.dim == 2:
            nx, ny = grid
            a = g.reshape(N, ny, p, nx, p).transpose(1, 3, 0, 2, 4)
        else:
            nx, ny, nz = grid
            a = g.reshape(N, nz, p, ny, p, nx, p).transpose(1, 3, 5, 0, 2, 4, 6)
        return np.ascontiguousarray(a).reshape(-1)


def periodic_grid(grid: tuple[int, ...]) -> np.ndarray:
    """Face neighbours of a periodic patch grid (x fastest)."""
    dim = len(grid)
    K = int(np.prod(grid))
    idx = np.arange(K).reshape(grid[::-1])  # [(nz,) ny, nx]
    nbr = np.zeros((K, 2 * dim), dtype=np.int32)
    for d in range(dim):
        ax = dim - 1 - d
        nbr[:, 2 * d] = np.roll(idx, 1, axis=ax).reshape(-1)      # -d neighbour
        nbr[:, 2 * d + 1] = np.roll(idx, -1, axis=ax).reshape(-1)  # +d neighbour
    return nbr


def self_periodic(K: int, dim: int) -> np.ndarray:
    return np.repeat(np.arange(K, dtype=np.int32)[:, None], 2 * dim, axis=1)


def _centres(grid_cells: tuple[int, ...], dx: float) -> list[np.ndarray]:
    """cell-centre coordinates x_i = (i + 1/2) dx per axis (x first)."""
    return [(np.arange(n, dtype=np.float64) + 0.5) * dx for n in grid_cells]


def euler_prim_to_state(rho, vel, p, gamma):
    """Euler IC in conserved variables: (rho, rho v, p/(gamma-1) + rho|v|^2/2)."""
    ke = 0.5 * rho * sum(v * v for v in vel)
    return [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]


# ---------------------------------------------------------------- configs --


def make_uniform_batch(grid, p, h, pde, params, N, dx):
    dim = len(grid)
    K = int(np.prod(grid))
    origin = np.zeros((K, dim))
    for k in range(K):
        r = k
        for d in range(dim):
            origin[k, d] = (r % grid[d]) * p * dx
            r //= grid[d]
    return Batch(dim=dim, p=np.full(K, p, np.int32), dx=np.full(K, dx), nbr=periodic_grid(grid),
                 halo=h, pde=pde, params=np.asarray(params, np.float64), n_unknowns=N,
                 state=np.zeros(K * p ** dim * N), origin=origin)


def config0(n_patch: int = 8, p: int = 8, gamma: float = 1.4) -> Batch:
    """2D Euler entropy wave on [0,1]^2, n_patch^2 patches of p^2 cells, h = 1."""
    n = n_patch * p
    dx = 1.0 / n
    b = make_uniform_batch((n_patch, n_patch), p, 1, "euler", [gamma], 4, dx)
    x, y = _centres((n, n), dx)
    X, Y = np.meshgrid(x, y, indexing="xy")  # [Y, X]
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    u = np.full_like(rho, 0.5)
    v = np.full_like(rho, 0.3)
    pr = np.ones_like(rho)
    g = np.stack(euler_prim_to_state(rho, [u, v], pr, gamma))
    b.state = b.from_global(g, (n_patch, n_patch))
    return b


C1_GRID = (16, 16, 8)


def fourier_field(seed: int, coords, lengths, n_modes: int = 8, kmax: int = 4) -> np.ndarray:
    """sum_m A_m sin(2 pi k_m . x/L + phi_m) / sum_m A_m on a tensor grid,
    k_m in {-kmax..kmax}^3 minus 0, A_m ~ U(0,1), phi_m ~ U(0, 2 pi)."""
    nk = 2 * kmax + 1
    r = uniform(seed, 3 * n_modes)
    kidx = splitmix64(substream(seed, 1), n_modes) % np.uint64(nk ** 3 - 1)
    kidx = kidx.astype(np.int64)
    kidx = np.where(kidx >= (nk ** 3 - 1) // 2, kidx + 1, kidx)  # skip k = 0
    nz, ny, nx = len(coords[2]), len(coords[1]), len(coords[0])
    out = np.zeros((nz, ny, nx))
    tmp = np.empty((nz, ny, nx))
    asum = 0.0
    for m in range(n_modes):
        kk = [int(kidx[m] % nk) - kmax, int((kidx[m] // nk) % nk) - kmax, int(kidx[m] // nk ** 2) - kmax]
        A = r[3 * m]
        phi = 2 * np.pi * r[3 * m + 1]
        # sin(u(z) + w(y, x)) = sin u cos w + cos u sin w, evaluated separably
        u = phi + (2 * np.pi * kk[2] / lengths[2]) * coords[2]
        w = ((2 * np.pi * kk[1] / lengths[1]) * coords[1])[:, None] + \
            ((2 * np.pi * kk[0] / lengths[0]) * coords[0])[None, :]
        np.multiply((A * np.sin(u))[:, None, None], np.cos(w)[None], out=tmp)
        out += tmp
        np.multiply((A * np.cos(u))[:, None, None], np.sin(w)[None], out=tmp)
        out += tmp
        asum += A
    return out / asum


def config1(seed: int = 1, grid=C1_GRID, p: int = 16, gamma: float = 1.4, halo: int = 1) -> Batch:
    """3D Euler, smooth random IC (sum of 8 Fourier modes per primitive).
    halo = 1 for the finite-volume step, 3 for the FD4 + KO6 step."""
    cells = tuple(g * p for g in grid)
    dx = 1.0 / cells[0]
    b = make_uniform_batch(grid, p, halo, "euler", [gamma], 5, dx)
    lengths = tuple(c * dx for c in cells)
    coords = _centres(cells, dx)
    s = [fourier_field(substream(seed, 10 + f), coords, lengths) for f in range(5)]
    rho = 1.0 + 0.5 * s[0]
    pr = 1.0 + 0.5 * s[4]
    vs = 0.49 / math.sqrt(3.0)
    vel = [vs * s[1], vs * s[2], vs * s[3]]
    g = np.stack(euler_prim_to_state(rho, vel, pr, gamma))
    b.state = b.from_global(g, grid)
    return b


def adv_var_batch(grid, p: int, kappa: float = 0.0, field: str = "random", seed: int = 31, halo: int = 1,
                  q0=None) -> Batch:
    """Linear advection with a velocity field carried as material parameters:
    per cell (q, a_x, a_y(, a_z)) on a periodic patch grid over [0,1)^dim.
    field "random": every a_d varies in every direction (compressive);
    "shear": a_d does not depend on x_d (discretely divergence-free);
    "const": a = (0.6, -0.3, 0.2).  q defaults to 1 + sin(2 pi x) cos(2 pi y)/2."""
    dim = len(grid)
    cells = tuple(g * p for g in grid)
    dx = 1.0 / cells[0]
    b = make_uniform_batch(grid, p, halo, "adv_var", [kappa], 1 + dim, dx)
    c = _centres(cells, dx)
    if dim == 3:
        Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    else:
        Y, X = np.meshgrid(c[1], c[0], indexing="ij")
        Z = np.zeros_like(X)
    ph = 2 * np.pi * uniform(seed, 6)
    tp = 2 * np.pi
    if field == "random":
        a = [0.5 + 0.3 * np.sin(tp * Y + ph[0]) + 0.2 * np.sin(tp * X + ph[1]) + 0.1 * np.cos(tp * Z + ph[2]),
             -0.3 + 0.3 * np.cos(tp * X + ph[3]) + 0.2 * np.sin(tp * Y + ph[4]),
             0.2 + 0.25 * np.sin(tp * (X + Z) + ph[5])]
    elif field == "shear":
        a = [0.5 + 0.3 * np.sin(tp * Y + ph[0]) + 0.1 * np.cos(tp * Z + ph[2]),
             -0.3 + 0.3 * np.cos(tp * X + ph[3]) + 0.1 * np.sin(tp * Z + ph[1]),
             0.2 + 0.25 * np.sin(tp * (X + Y) + ph[5])]
    else:
        a = [np.full_like(X, 0.6), np.full_like(X, -0.3), np.full_like(X, 0.2)]
    q = 1.0 + 0.5 * np.sin(tp * X) * np.cos(tp * Y) if q0 is None else q0(X, Y, Z)
    b.state = b.from_global(np.stack([q] + a[:dim]), grid)
    return b


def independent_euler_patches(seed: int, K: int, p: int, halo: int = 1, gamma: float = 1.4) -> Batch:
    """K independent 3D Euler patches of p^3 cells (each periodic on itself,
    dx = 1/p), i.i.d. primitives per cell: rho, p ~ U[0.8, 1.2], each
    velocity component ~ U[-0.3, 0.3].  The batch shape of the K sweep
    (many small patches handed over at once, each with its own halo)."""
    n = K * p ** 3
    rho = uniform(substream(seed, 1), n, 0.8, 1.2)
    vel = [uniform(substream(seed, 2 + d), n, -0.3, 0.3) for d in range(3)]
    pr = uniform(substream(seed, 5), n, 0.8, 1.2)
    cons = np.stack(euler_prim_to_state(rho, vel, pr, gamma))            # [5, K p^3]
    state = np.ascontiguousarray(cons.reshape(5, K, p ** 3).transpose(1, 0, 2)).reshape(-1)
    return Batch(dim=3, p=np.full(K, p, np.int32), dx=np.full(K, 1.0 / p), nbr=self_periodic(K, 3), halo=halo,
                 pde="euler", params=np.array([gamma]), n_unknowns=5, state=state)


def _unit_cube_modes(seed: int, K: int, p: int, n_modes: int) -> np.ndarray:
    """[K, p^3] per patch: sum_m a_m sin(2 pi k_m . x + phi_m) / sum_m a_m
    at the cell centres of the unit cube (x fastest), k_m in {-1,0,1}^3
    minus 0, a_m ~ U(0,1), phi_m ~ U(0, 2 pi); values in [-1, 1]."""
    x = (np.arange(p) + 0.5) / p
    e = np.exp(2j * np.pi * np.outer(np.arange(-1, 2), x))            # e[k+1, i]
    r = uniform(seed, K * n_modes * 2).reshape(K, n_modes, 2)
    kk = (splitmix64(substream(seed, 5), K * n_modes) % np.uint64(26)).astype(np.int64).reshape(K, n_modes)
    kk = np.where(kk >= 13, kk + 1, kk)  # skip (0,0,0), index 13 of 27
    kx, ky, kz = kk % 3, (kk // 3) % 3, kk // 9
    amp = r[:, :, 0] * np.exp(1j * 2 * np.pi * r[:, :, 1])            # [K, m]
    out = np.zeros((K, p, p, p))
    for m in range(n_modes):
        t = amp[:, m, None, None, None] * e[kz[:, m]][:, :, None, None] * e[ky[:, m]][:, None, :, None] \
            * e[kx[:, m]][:, None, None, :]
        out += np.imag(t)
    return out.reshape(K, p ** 3) / r[:, :, 0].sum(axis=1)[:, None]


def independent_euler_patches_smooth(seed: int, K: int, p: int, halo: int = 1, gamma: float = 1.4) -> Batch:
    """K independent 3D Euler patches of p^3 cells (each a periodic unit cube
    on itself, dx = 1/p) with a smooth seeded state: per patch a uniform
    velocity v_k (components ~ U[-0.3, 0.3]) carrying an entropy wave
    rho = 1 + 0.2 s_rho, plus small acoustic perturbations v = v_k + 0.02 s_v,
    p = 1 + 0.02 s_p, each s a normalised sum of 4 modes with wave vectors in
    {-1,0,1}^3.  Stays smooth (far from shock formation) for the several
    hundred FD4 + KO6 + RK4 steps of the K sweep, unlike i.i.d. cell values,
    which the unlimited central scheme cannot carry."""
    fields = [_unit_cube_modes(substream(seed, 20 + f), K, p, 4) for f in range(5)]
    vk = uniform(substream(seed, 30), 3 * K, -0.3, 0.3).reshape(3, K)
    rho = 1.0 + 0.2 * fields[0]
    vel = [vk[d][:, None] + 0.02 * fields[1 + d] for d in range(3)]
    pr = 1.0 + 0.02 * fields[4]
    cons = np.stack(euler_prim_to_state(rho, vel, pr, gamma))            # [5, K, p^3]
    state = np.ascontiguousarray(cons.transpose(1, 0, 2)).reshape(-1)
    return Batch(dim=3, p=np.full(K, p, np.int32), dx=np.full(K, 1.0 / p), nbr=self_periodic(K, 3), halo=halo,
                 pde="euler", params=np.array([gamma]), n_unknowns=5, state=state)


def independent_halo_chunks(seed: int, K: int, p: int, halo: int = 1, gamma: float = 1.4) -> list:
    """K offload-mode input chunks of 3D Euler: each the (p+2h)^3 halo box in
    per-point order [z][y][x][5], i.i.d. primitives at every point (halo
    included: in offload mode the caller supplies the halo values):
    rho, p ~ U[0.8, 1.2], velocity components ~ U[-0.3, 0.3]."""
    pb = p + 2 * halo
    n = K * pb ** 3
    rho = uniform(substream(seed, 1), n, 0.8, 1.2)
    vel = [uniform(substream(seed, 2 + d), n, -0.3, 0.3) for d in range(3)]
    pr = uniform(substream(seed, 5), n, 0.8, 1.2)
    cons = np.stack(euler_prim_to_state(rho, vel, pr, gamma), axis=-1)      # [n, 5]
    return [np.ascontiguousarray(c) for c in cons.reshape(K, pb, pb, pb, 5)]


# ------------------------------------------------------------------- SRHD --


def srhd_primitives(seed: int, n: int):
    """i.i.d. SRHD primitives: rho, eps log-uniform in [1e-3, 10], W ~ U[1,10],
    isotropic direction.  Returns (rho, vx, vy, vz, eps)."""
    u = uniform(seed, 5 * n).reshape(5, n)
    lo, hi = math.log(1e-3), math.log(10.0)
    rho = np.exp(lo + (hi - lo) * u[0])
    eps = np.exp(lo + (hi - lo) * u[1])
    W = 1.0 + 9.0 * u[2]
    vmag = np.sqrt(1.0 - 1.0 / (W * W))
    ct = 2.0 * u[3] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * u[4]
    return rho, vmag * st * np.cos(ph), vmag * st * np.sin(ph), vmag * ct, eps


def srhd_prim_to_cons(rho, vx, vy, vz, eps, Gam):
    """D = rho W, S = rho h W^2 v, tau = rho h W^2 - p - D, p = (Gamma-1) rho eps,
    h = 1 + eps + p/rho (the inverse map is what the library recovers)."""
    p = (Gam - 1.0) * rho * eps
    W = 1.0 / np.sqrt(1.0 - (vx * vx + vy * vy + vz * vz))
    h = 1.0 + eps + p / rho
    rhW2 = rho * h * W * W
    return np.stack([rho * W, rhW2 * vx, rhW2 * vy, rhW2 * vz, rhW2 - p - rho * W]), p


def config3(seed: int = 3, grid=C1_GRID, p: int = 16, Gam: float = 5.0 / 3.0,
            tol: float = 1e-12, maxit: int = 50) -> Batch:
    cells = tuple(g * p for g in grid)
    dx = 1.0 / cells[0]
    b = make_uniform_batch(grid, p, 1, "srhd", [Gam, tol, maxit], 5, dx)
    n = b.total_cells
    rho, vx, vy, vz, eps = srhd_primitives(seed, n)
    cons, _ = srhd_prim_to_cons(rho, vx, vy, vz, eps, Gam)
    # i.i.d. per cell: the draw order is the exchange-layout cell order
    K = b.K
    C = p ** 3
    b.state = np.ascontiguousarray(cons.reshape(5, K, C).transpose(1, 0, 2)).reshape(-1)
    return b


def srhd_training_pairs(seed: int, n: int, Gam: float = 5.0 / 3.0):
    """(cons [5, n], p [n]) pairs over the config-3 primitive ranges."""
    rho, vx, vy, vz, eps = srhd_primitives(seed, n)
    cons, p = srhd_prim_to_cons(rho, vx, vy, vz, eps, Gam)
    return cons, p


# -------------------------------------------------------- linear system --


def linsym_matrices(seed: int, N: int = 58, dim: int = 3):
    """B_d = A_d / rho(A_d), A_d = (G + G^T)/2, G_ij ~ N(0,1)."""
    Bs, rhos = [], []
    for d in range(dim):
        G = normal(substream(seed, 100 + d), N * N).reshape(N, N)
        A = 0.5 * (G + G.T)
        r = float(np.max(np.abs(np.linalg.eigvalsh(A))))
        B = A / r
        Bs.append(B)
        rhos.append(float(np.max(np.abs(np.linalg.eigvalsh(B)))))
    return np.stack(Bs), rhos


def linsym_params(Bs, rhos):
    dim = Bs.shape[0]
    rr = list(rhos) + [0.0] * (3 - dim)
    return np.concatenate([np.asarray(rr, np.float64), Bs.reshape(-1)])


def config2_sizes(seed: int = 2, n_patches: int = 4096):
    """Patch sizes 4, 8, 16 in exact ratio 1:2:1, shuffled (Fisher-Yates on
    SplitMix64)."""
    q = n_patches // 4
    sizes = np.array([4] * q + [8] * (n_patches - 2 * q) + [16] * q, dtype=np.int32)
    r = splitmix64(substream(seed, 7), n_patches)
    for i in range(n_patches - 1, 0, -1):
        j = int(r[i] % np.uint64(i + 1))
        sizes[i], sizes[j] = sizes[j], sizes[i]
    return sizes


def _linsym_modes(seed: int, k: int, N: int, n_modes: int):
    """mode parameters of patch k: complex amplitudes a e^{i phi} [N, m] and
    wave vectors (kx, ky, kz) [N, m] in {-1,0,1}^3 minus 0, a ~ U(-1/4, 1/4)"""
    s = substream(seed, 1000 + k)
    r = uniform(s, N * n_modes * 3).reshape(N, n_modes, 3)
    kk = (splitmix64(substream(s, 5), N * n_modes) % np.uint64(26)).astype(np.int64).reshape(N, n_modes)
    kk = np.where(kk >= 13, kk + 1, kk)  # skip (0,0,0), index 13 of 27
    amp = (-0.25 + 0.5 * r[:, :, 0]) * np.exp(1j * 2 * np.pi * r[:, :, 1])
    return amp, kk % 3 - 1, (kk // 3) % 3 - 1, kk // 9 - 1


def linsym_patches_ic(seed: int, ks, p: int, N: int, n_modes: int = 4) -> np.ndarray:
    """[len(ks), N, p, p, p] IC of patches ks (all of size p): per unknown the
    sum of n_modes terms a sin(2 pi k.x + phi) on the unit cube at cell centres,
    evaluated separably as Im(a e^{i phi} e^{2 pi i kz z} e^{2 pi i ky y} e^{2 pi i kx x})."""
    import torch  # multithreaded elementwise products on the host
    x = (np.arange(p) + 0.5) / p
    e = torch.from_numpy(np.exp(2j * np.pi * np.outer(np.arange(-1, 2), x)))  # e[k+1, i] = exp(2 pi i k x_i)
    G = len(ks)
    out = torch.zeros((G, N, p, p, p), dtype=torch.float64)
    params = [_linsym_modes(seed, int(k), N, n_modes) for k in ks]
    amp = torch.from_numpy(np.stack([q[0] for q in params]))            # [G, N, m]
    kx = torch.from_numpy(np.stack([q[1] for q in params]) + 1)
    ky = torch.from_numpy(np.stack([q[2] for q in params]) + 1)
    kz = torch.from_numpy(np.stack([q[3] for q in params]) + 1)
    for m in range(n_modes):
        az = amp[:, :, m, None] * e[kz[:, :, m]]     # [G, N, p]
        exy = e[ky[:, :, m]][:, :, :, None] * e[kx[:, :, m]][:, :, None, :]   # [G, N, p, p]
        out += torch.imag(az[:, :, :, None, None] * exy[:, :, None, :, :])
    return out.numpy()


def linsym_patch_ic(seed: int, k: int, p: int, N: int, n_modes: int = 4) -> np.ndarray:
    """[N, p, p, p] IC of patch k (see linsym_patches_ic)"""
    return linsym_patches_ic(seed, [k], p, N, n_modes)[0]


def config2(seed: int = 2, n_patches: int = 4096, subset=None, N: int = 58,
            sizes=None, h: int = 3) -> Batch:
    """Uneven batch of independent periodic unit-cube patches.  `subset`
    selects patch indices of the full shuffled batch (the IC of a patch depends
    only on (seed, its index), so a subset equals those patches of the full
    batch)."""
    if sizes is None:
        sizes = config2_sizes(seed, n_patches)
    idx = np.arange(len(sizes)) if subset is None else np.asarray(subset)
    ps = sizes[idx].astype(np.int32)
    K = len(ps)
    Bs, rhos = linsym_matrices(seed, N)
    C = ps.astype(np.int64) ** 3
    off = np.concatenate([[0], np.cumsum(C)]) * N
    state = np.empty(int(off[-1]))
    for p in np.unique(ps):
        pos = np.nonzero(ps == p)[0]
        step = max(1, 65536 // int(p) ** 3)
        for c0 in range(0, len(pos), step):
            chunk = pos[c0:c0 + step]
            blocks = linsym_patches_ic(seed, idx[chunk], int(p), N)
            for j, blk in zip(chunk, blocks):
                state[off[j]:off[j + 1]] = blk.reshape(-1)
    return Batch(dim=3, p=ps, dx=1.0 / ps.astype(np.float64), nbr=self_periodic(K, 3), halo=h,
                 pde="linsym", params=linsym_params(Bs, rhos), n_unknowns=N, state=state)


def config2_subset(seed: int = 2, n_per_size=(16, 16, 16)):
    """Seeded subset of the full config-2 batch covering every patch size."""
    sizes = config2_sizes(seed)
    sel = []
    for ps, cnt in zip((4, 8, 16), n_per_size):
        where = np.nonzero(sizes == ps)[0]
        pick = splitmix64(substream(seed, 11, ps), cnt) % np.uint64(len(where))
        chosen = []
        for v in pick.astype(np.int64):
            j = int(v)
            while where[j] in chosen:
                j = (j + 1) % len(where)
            chosen.append(int(where[j]))
        sel += chosen
    return sorted(sel)


# ------------------------------------------------------ training batches --


def feistel_permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """The seeded permutation of [0, n) that orders the training rows of one
    epoch: a balanced four-round Feistel network on 2h bits (h the smallest
    value with 2^(2h) >= n, 2h >= 2) with cycle walking into [0, n) (Black &
    Rogaway, "Ciphers with arbitrary finite domains", CT-RSA 2002).  Key =
    mix(seed + (epoch + 1) G), round r (0..3): L, R <- R, L ^ (mix(key ^
    (r + 1) G ^ R) & (2^h - 1)), value L 2^h + R; mix is the SplitMix64
    finaliser, G = 0x9E3779B97F4A7C15.  Returns int64 [n]."""
    if n == 0:
        return np.zeros(0, np.int64)
    m = 2
    while m < 62 and (1 << m) < n:
        m += 1
    h = (m + 1) // 2
    mask = np.uint64((1 << h) - 1)
    with np.errstate(over="ignore"):
        key = _mix(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + np.uint64(epoch + 1) * _GOLDEN],
                            dtype=np.uint64))[0]
        rk = [key ^ (np.uint64(r + 1) * _GOLDEN) for r in range(4)]

        def perm(v):
            L, R = v >> np.uint64(h), v & mask
            for r in range(4):
                f = _mix(rk[r] ^ R) & mask
                L, R = R, L ^ f
            return (L << np.uint64(h)) | R

        v = perm(np.arange(n, dtype=np.uint64))
        todo = v >= np.uint64(n)
        while todo.any():
            v[todo] = perm(v[todo])
            todo = v >= np.uint64(n)
    return v.astype(np.int64)
