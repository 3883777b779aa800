"""poisson.py -- TEST INFRASTRUCTURE: reference electrostatic initial field.

The discrete Poisson equation of Section 4.3 (Eq. poiphi) on the periodic
grid, for the cell-centred potential Phi of a cell-centred charge density
rho:

    sum_a (-Phi_{c-e_a} + 2 Phi_c - Phi_{c+e_a}) / d_a^2 = 4 pi rho_c,

solved exactly by the discrete Fourier transform (a library FFT; the
operator's eigenvalue for wave numbers k is sum_a (2 - 2 cos(2 pi k_a /
N_a)) / d_a^2), with the k = 0 mode of rho removed (a uniform background of
the opposite charge) and Phi of zero mean.  The face-centred field follows
from Eq. egradphidis: E^x at face i (between cells i-1 and i) is
(Phi_{i-1} - Phi_i) / dx, and likewise for y and z.  Only the tests use this
module; it shares no code with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np


def solve(grid, rho: np.ndarray):
    """Phi (nz, ny, nx) of rho minus its mean; grid has nx, ny, nz, dx, dy, dz."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = (grid.nz, grid.ny, grid.nx)
    assert rho.shape == shape
    lam = np.zeros(shape)
    for axis, (n, h) in enumerate(((grid.nz, grid.dz), (grid.ny, grid.dy), (grid.nx, grid.dx))):
        k = np.arange(n)
        e = (2.0 - 2.0 * np.cos(2.0 * math.pi * k / n)) / (h * h)
        sh = [1, 1, 1]
        sh[axis] = n
        lam = lam + e.reshape(sh)
    rhat = np.fft.fftn(rho - rho.mean())
    phat = np.zeros_like(rhat)
    nz = lam != 0.0
    phat[nz] = 4.0 * math.pi * rhat[nz] / lam[nz]
    return np.real(np.fft.ifftn(phat))


def e_of_phi(grid, phi: np.ndarray) -> np.ndarray:
    """E (3, nz, ny, nx) on the faces from the cell-centred potential (Eq.
    egradphidis)."""
    E = np.zeros((3,) + phi.shape)
    E[0] = (np.roll(phi, 1, axis=2) - phi) / grid.dx
    E[1] = (np.roll(phi, 1, axis=1) - phi) / grid.dy
    E[2] = (np.roll(phi, 1, axis=0) - phi) / grid.dz
    return E


def div_e(grid, E: np.ndarray) -> np.ndarray:
    """Cell-centred divergence of the face field (the discrete Gauss law's left side)."""
    return ((np.roll(E[0], -1, axis=2) - E[0]) / grid.dx + (np.roll(E[1], -1, axis=1) - E[1]) / grid.dy
            + (np.roll(E[2], -1, axis=0) - E[2]) / grid.dz)
