"""Seeded synthetic plasma inputs shared by the oracle tests, the GPU tests and
the benchmark.

This module only draws initial states (positions, momenta, weights) and
states the workload parameters; it holds none of the PIC method's arithmetic.
Every draw comes from ``numpy.random.Generator(PCG64(seed))`` in a fixed order
(positions x, y, z for all particles, then momenta), so the oracle and the GPU
library receive bit-identical inputs.

Units: Gaussian, c = 1 unless stated, dx = dy = dz = 1 (V = 1), positions in
cell units, momenta as w = gamma v in units of c.  Electrons carry charge
-W and mass W per macro-particle, with the weight W chosen so that the mean
electron density gives the requested plasma frequency:
omega_pe^2 = 4 pi (ppc / V) W  ->  W = omega_pe^2 V / (4 pi ppc).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

BASE_SEED = 11010809


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dims: int              # 2: 2D3V (nz == 1, no z dependence), 3: 3D3V
    dt: float
    ppc: int               # electrons per cell (per occupied cell for slabs)
    w_th: tuple            # thermal momentum spread per axis (units of c)
    omega_pe: float
    steps: int
    sort_every: int = 0
    drift: float = 0.0     # +-drift along x for two counter-streaming halves
    bext: tuple = (0.0, 0.0, 0.0)
    slab: tuple = None     # (x_lo, x_hi): electrons only in this x range
    ions_mobile: bool = False
    ion_mass: float = 100.0
    ion_w_th: float = 0.005
    source: tuple = None   # (plane, amplitude, omega, ramp time): +x E^y plane wave
    xbc: str = "periodic"  # x boundary: "periodic", or "open" (absorbing walls)
    seed: int = BASE_SEED

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def occupied_cells(self) -> int:
        if self.slab is None:
            return self.ncell
        return (self.slab[1] - self.slab[0]) * self.ny * self.nz

    @property
    def n_electrons(self) -> int:
        return self.ppc * self.occupied_cells

    @property
    def n_particles(self) -> int:
        """Mobile particles: the electrons, plus as many ions when they move."""
        return self.n_electrons * (2 if self.ions_mobile else 1)

    @property
    def weight(self) -> float:
        return self.omega_pe ** 2 / (4.0 * math.pi * self.ppc)

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five benchmark configurations (names describe the workload).  Where the
# workload statement is silent the readings listed in the design notes apply:
# omega_pe = w_th / dx (Debye length one cell), co-located immobile ions.
WORKLOADS = {
    "2d3v_32x32_fp64": Workload("2d3v_32x32_fp64", 32, 32, 1, 2, 0.5, 4, (0.05,) * 3, 0.05,
                                100, seed=BASE_SEED + 1),
    "3d_64cube_8ppc": Workload("3d_64cube_8ppc", 64, 64, 64, 3, 0.45, 8, (0.1,) * 3, 0.1, 50,
                               sort_every=10, seed=BASE_SEED + 2),
    "3d_128cube_slab": Workload("3d_128cube_slab", 128, 128, 128, 3, 0.45, 16, (0.01,) * 3,
                                0.1 * 2 * math.pi / 20.0, 200, sort_every=10, slab=(32, 96),
                                source=(8, 2 * math.pi / 20.0, 2 * math.pi / 20.0, 20.0),
                                xbc="open", seed=BASE_SEED + 3),
    "2d3v_256sq_beams": Workload("2d3v_256sq_beams", 256, 256, 1, 2, 0.5, 16, (0.02,) * 3, 0.02,
                                 200, drift=0.2, bext=(0.0, 0.0, 0.02), sort_every=20,
                                 seed=BASE_SEED + 4),
    "3d_256cube_weibel": Workload("3d_256cube_weibel", 256, 256, 256, 3, 0.45, 32,
                                  (0.3, 0.05, 0.05), 0.05, 100, sort_every=20,
                                  ions_mobile=True, seed=BASE_SEED + 5),
}


@dataclass
class Plasma:
    """Initial electron state: x (3, n), w (3, n), weight (n,), all float64."""
    x: np.ndarray
    w: np.ndarray
    weight: np.ndarray
    q: float = -1.0
    m: float = 1.0

    @property
    def n(self) -> int:
        return self.weight.shape[0]


def electrons(wl: Workload, n: int = None, rng: np.random.Generator = None) -> Plasma:
    """Uniform random positions (inside the slab if any), Gaussian momenta of
    spread w_th per axis, +-drift along x on alternating halves."""
    n = wl.n_electrons if n is None else n
    rng = np.random.Generator(np.random.PCG64(wl.seed)) if rng is None else rng
    x = np.empty((3, n))
    lo_x, hi_x = (0.0, float(wl.nx)) if wl.slab is None else (float(wl.slab[0]), float(wl.slab[1]))
    x[0] = rng.uniform(lo_x, hi_x, n)
    x[1] = rng.uniform(0.0, float(wl.ny), n)
    x[2] = rng.uniform(0.0, float(wl.nz), n)
    w = np.empty((3, n))
    for a in range(3):
        w[a] = rng.normal(0.0, wl.w_th[a], n)
    if wl.drift:
        w[0, : n // 2] += wl.drift
        w[0, n // 2:] -= wl.drift
    # positions are in [lo, hi); guard against the open upper end
    for a, top in enumerate((hi_x, float(wl.ny), float(wl.nz))):
        x[a] = np.where(x[a] >= top, 0.0, x[a])
    return Plasma(x, w, np.full(n, wl.weight))


def ions_like(wl: Workload, e: Plasma, rng: np.random.Generator = None) -> Plasma:
    """Ions co-located with the electrons (so the initial charge density is
    zero everywhere), charge +W and mass ion_mass * W; momenta Gaussian with
    spread ion_w_th when the ions are mobile, zero otherwise."""
    w = np.zeros_like(e.w)
    if wl.ions_mobile:
        rng = np.random.Generator(np.random.PCG64(wl.seed + 1000)) if rng is None else rng
        w = rng.normal(0.0, wl.ion_w_th, e.w.shape)
    return Plasma(e.x.copy(), w, e.weight.copy(), q=1.0, m=wl.ion_mass)


def lattice_electrons(wl: Workload, drift=(0.0, 0.0, 0.0)) -> Plasma:
    """Cold electrons placed on ppc sub-lattices of unit spacing, every one with
    the same momentum ``drift``; sub-lattice offsets are fixed, not random."""
    k = max(1, round(wl.ppc ** (1.0 / wl.dims)))
    offs = (np.arange(k) + 0.5) / k
    if wl.dims == 2:
        ox, oy = np.meshgrid(offs, offs, indexing="ij")
        sub = np.stack([ox.ravel(), oy.ravel(), np.full(ox.size, 0.5)])
    else:
        ox, oy, oz = np.meshgrid(offs, offs, offs, indexing="ij")
        sub = np.stack([ox.ravel(), oy.ravel(), oz.ravel()])
    ci, cj, ck = np.meshgrid(np.arange(wl.nx), np.arange(wl.ny), np.arange(wl.nz), indexing="ij")
    cells = np.stack([ci.ravel(), cj.ravel(), ck.ravel()]).astype(np.float64)
    x = (cells[:, :, None] + sub[:, None, :]).reshape(3, -1)
    n = x.shape[1]
    w = np.tile(np.asarray(drift, dtype=np.float64)[:, None], (1, n))
    weight = np.full(n, wl.omega_pe ** 2 / (4.0 * math.pi * sub.shape[1]))
    return Plasma(np.ascontiguousarray(x), w, weight)


def random_moves(n: int, seed: int, box=(16, 16, 16), max_step=0.9):
    """Random particle start points inside a box and displacements of at most
    ``max_step`` cells per axis (a kernel or oracle test input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.stack([rng.uniform(0, box[a], n) for a in range(3)])
    dx = rng.uniform(-max_step, max_step, (3, n))
    return x0, x0 + dx


def beams(box, n: int, seed: int, w_th: float = 0.1, drift: float = 0.0, dims: int = 3):
    """Small differentiable test plasma: n electrons at uniform random
    positions in box = (nx, ny, nz), Gaussian momenta of spread w_th per axis,
    +drift / -drift along x on the two halves, weights giving
    omega_pe = w_th at the mean density.  dims == 2 puts every particle on
    z = 0.  Returns (x, w, weight)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.stack([rng.uniform(0, box[a], n) for a in range(3)])
    w = rng.normal(0.0, w_th, (3, n))
    w[0, : n // 2] += drift
    w[0, n // 2:] -= drift
    ppc = n / (box[0] * box[1] * box[2])
    weight = np.full(n, w_th ** 2 / (4 * math.pi * ppc))
    if dims == 2:
        x[2] = 0.0
    return x, w, weight


def device_chunks(wl: Workload, device, chunk: int = 1 << 26, ions: bool = False):
    """Yield (x, w, weight) torch float64 tensors on ``device`` covering the
    whole species in chunks of ``chunk`` particles, drawn with
    ``torch.Generator(device)`` seeded by (workload seed, chunk index) -- for
    workloads too large to draw on the host.  Same distributions as
    ``electrons`` / ``ions_like``; ions (``ions=True``) are co-located with the
    electrons of the same chunk (same position draws)."""
    import torch

    n = wl.n_electrons
    lo_x, hi_x = (0.0, float(wl.nx)) if wl.slab is None else (float(wl.slab[0]), float(wl.slab[1]))
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        gen = torch.Generator(device=device)
        gen.manual_seed(wl.seed * 1000003 + c0 // chunk)
        u = torch.rand((3, m), generator=gen, dtype=torch.float64, device=device)
        x = torch.empty((3, m), dtype=torch.float64, device=device)
        x[0] = lo_x + (hi_x - lo_x) * u[0]
        x[1] = float(wl.ny) * u[1]
        x[2] = float(wl.nz) * u[2]
        del u
        tops = torch.tensor([hi_x, float(wl.ny), float(wl.nz)], dtype=torch.float64,
                            device=device)[:, None]
        x = torch.where(x >= tops, torch.zeros_like(x), x)
        if ions:
            gi = torch.Generator(device=device)
            gi.manual_seed(wl.seed * 1000003 + 7919 + c0 // chunk)
            if wl.ions_mobile:
                w = wl.ion_w_th * torch.randn((3, m), generator=gi, dtype=torch.float64,
                                              device=device)
            else:
                w = torch.zeros((3, m), dtype=torch.float64, device=device)
        else:
            w = torch.randn((3, m), generator=gen, dtype=torch.float64, device=device)
            for a in range(3):
                w[a] *= wl.w_th[a]
            if wl.drift:
                w[0, : m // 2] += wl.drift
                w[0, m // 2:] -= wl.drift
        yield x, w, torch.full((m,), wl.weight, dtype=torch.float64, device=device)
