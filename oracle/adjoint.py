"""adjoint.py -- TEST INFRASTRUCTURE: the reference gradient for the GPU adjoint.

A second plain FP64 CPU implementation of the particle-in-cell step of
Sokolov, arXiv:1101.0809 (the Appendix algorithm), written in PyTorch tensor
operations so that ``torch.autograd`` differentiates it exactly: the gradient
of the final field energy with respect to the initial momenta, the initial
positions and the external uniform magnetic field, and the vector-Jacobian
product of one step.  Only the tests use it; it shares no code
with the GPU path.  It follows the readings of the C oracle (``pic_oracle.c``)
and the tests check its forward step against that oracle, and its gradient
against central differences of that oracle.

Everything is the slow, obvious form, vectorised over particles only:
  * form factors as functions of the distance (Section 3.1, 4.5): node weight
    f^(1)(n - x), cell weight f^(2)(c + 1/2 - x), cumulative F (integral of
    f^(1));
  * gather (Eqs. alphax, betax) as a sum over a 5^3 box around floor(x);
  * push (Appendix, Eq. p2), position advance (Eq. coordscheme);
  * current in the one-sixth form of Eq. current over a 7^3 box around
    floor(x^n), which contains both end points' supports;
  * the Yee updates (Eqs. updateB, escheme);
  * loss: V/(8 pi) sum (E^N)^2 + (B^N)^2 with B^N the half-advanced field
    (the field energy of Section 4.1; the external B is not stored and is not
    part of it).
"""
from __future__ import annotations

import math

import numpy as np
from dataclasses import dataclass

import torch

DT = torch.float64


def f1(r):
    """Node weight f^(1)(r), the cap convolved once."""
    return torch.clamp(1.0 - r.abs(), min=0.0)


def f2(r):
    """Cell weight f^(2)(r), the cap convolved twice."""
    a = r.abs()
    return torch.where(a <= 0.5, 0.75 - a * a, torch.where(a < 1.5, 0.5 * (1.5 - a) ** 2, torch.zeros_like(a)))


def F1(s):
    """Integral of f^(1) from -infinity to s."""
    return torch.where(s <= -1.0, torch.zeros_like(s),
                       torch.where(s <= 0.0, 0.5 * (1.0 + s) ** 2,
                                   torch.where(s < 1.0, 1.0 - 0.5 * (1.0 - s) ** 2, torch.ones_like(s))))


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dt: float
    c: float = 1.0
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0

    @property
    def n(self):
        return (self.nx, self.ny, self.nz)

    @property
    def h(self):
        return (self.dx, self.dy, self.dz)

    @property
    def V(self):
        return self.dx * self.dy * self.dz


def _roll(a, shift, axis):
    """a shifted along a grid axis (0 = x, the last tensor dim); shift +1 gives a[i-1] at i."""
    return torch.roll(a, shifts=shift, dims=2 - axis)


def half_b(g: Grid, E, B):
    """B - (1/2) curl_h E (Eq. updateB): B^x at (i+1/2, j, k), B^y at (i, j+1/2, k), B^z at (i, j, k+1/2)."""
    cx, cy, cz = g.c * g.dt / g.dx, g.c * g.dt / g.dy, g.c * g.dt / g.dz
    Ex, Ey, Ez = E[0], E[1], E[2]
    Bx = B[0] - 0.5 * cy * (Ez - _roll(Ez, 1, 1)) + 0.5 * cz * (Ey - _roll(Ey, 1, 2))
    By = B[1] - 0.5 * cz * (Ex - _roll(Ex, 1, 2)) + 0.5 * cx * (Ez - _roll(Ez, 1, 0))
    Bz = B[2] - 0.5 * cx * (Ey - _roll(Ey, 1, 0)) + 0.5 * cy * (Ex - _roll(Ex, 1, 1))
    return torch.stack([Bx, By, Bz])


def update_e(g: Grid, E, B, J):
    """E - 4 pi dt J + curl_h B (Eq. escheme)."""
    cx, cy, cz = g.c * g.dt / g.dx, g.c * g.dt / g.dy, g.c * g.dt / g.dz
    f = 4.0 * math.pi * g.dt
    Bx, By, Bz = B[0], B[1], B[2]
    Ex = E[0] - f * J[0] + cy * (_roll(Bz, -1, 1) - Bz) - cz * (_roll(By, -1, 2) - By)
    Ey = E[1] - f * J[1] + cz * (_roll(Bx, -1, 2) - Bx) - cx * (_roll(Bz, -1, 0) - Bz)
    Ez = E[2] - f * J[2] + cx * (_roll(By, -1, 0) - By) - cy * (_roll(Bx, -1, 1) - Bx)
    return torch.stack([Ex, Ey, Ez])


def _flat(g: Grid, i, j, k):
    return (torch.remainder(k, g.nz) * g.ny + torch.remainder(j, g.ny)) * g.nx + torch.remainder(i, g.nx)


def gather(g: Grid, E, Bh, x, bext):
    """E with alpha^x = f_i(x) dF_j(y) dF_k(z) (Eq. alphax) and B^n with
    beta^x = dF_i(x) f_j(y) f_k(z) (Eq. betax), cyclic; plus the external B."""
    n = x.shape[1]
    base = torch.floor(x.detach()).to(torch.int64)
    o = torch.arange(-2, 3, dtype=torch.int64)
    nodes = base[:, None, :] + o[None, :, None]           # (3, 5, n)
    nw = f1(nodes.to(DT) - x[:, None, :])                 # node weights
    cw = f2(nodes.to(DT) + 0.5 - x[:, None, :])           # cell weights
    I = nodes[0][:, None, None, :]
    Jj = nodes[1][None, :, None, :]
    K = nodes[2][None, None, :, :]
    idx = _flat(g, I, Jj, K)                              # (5, 5, 5, n)

    def w3(wx, wy, wz):
        return wx[:, None, None, :] * wy[None, :, None, :] * wz[None, None, :, :]

    Ef, Bf = E.reshape(3, -1), Bh.reshape(3, -1)
    Ep = torch.stack([(w3(nw[0], cw[1], cw[2]) * Ef[0][idx]).sum((0, 1, 2)),
                      (w3(cw[0], nw[1], cw[2]) * Ef[1][idx]).sum((0, 1, 2)),
                      (w3(cw[0], cw[1], nw[2]) * Ef[2][idx]).sum((0, 1, 2))])
    Bp = torch.stack([(w3(cw[0], nw[1], nw[2]) * Bf[0][idx]).sum((0, 1, 2)),
                      (w3(nw[0], cw[1], nw[2]) * Bf[1][idx]).sum((0, 1, 2)),
                      (w3(nw[0], nw[1], cw[2]) * Bf[2][idx]).sum((0, 1, 2))])
    return Ep, Bp + bext[:, None]


def push(qm, dt, c, Ep, Bp, w):
    """Appendix: e = q dt E/(2m); w~ = w + e; b = q dt B/(2 m sqrt(w~^2 + c^2));
    w' = w~ + w~ x b; w_new = w~ + e + 2 (w' x b)/(1 + b^2)."""
    e = 0.5 * qm * dt * Ep
    wt = w + e
    gam = torch.sqrt((wt * wt).sum(0) + c * c)
    b = 0.5 * qm * dt * Bp / gam
    wp = wt + torch.cross(wt, b, dim=0)
    b2 = (b * b).sum(0)
    return wt + e + 2.0 * torch.cross(wp, b, dim=0) / (1.0 + b2)


def displacement(g: Grid, w):
    gam = torch.sqrt((w * w).sum(0) + g.c * g.c)
    h = torch.tensor(g.h, dtype=DT)[:, None]
    return (w / gam) * (g.c * g.dt / h)


def deposit(g: Grid, x0, x1, charge):
    """J of particles moving x0 -> x1 (x1 unwrapped), one-sixth form of Eq. current:
    xi^x = -(1/6)(dx/dt)[F_i(x1) - F_i(x0)] {2[dF_j(y1)dF_k(z1) + dF_j(y0)dF_k(z0)]
           + dF_j(y1)dF_k(z0) + dF_j(y0)dF_k(z1)}, cyclic; J += (q/V) xi."""
    nc = g.nx * g.ny * g.nz
    base = torch.floor(x0.detach()).to(torch.int64)
    o = torch.arange(-3, 4, dtype=torch.int64)
    nodes = base[:, None, :] + o[None, :, None]           # (3, 7, n)
    nd = nodes.to(DT)
    dF = F1(nd - x1[:, None, :]) - F1(nd - x0[:, None, :])
    s0 = f2(nd + 0.5 - x0[:, None, :])
    s1 = f2(nd + 0.5 - x1[:, None, :])
    J = []
    for comp in range(3):
        u, v = (comp + 1) % 3, (comp + 2) % 3
        brace = (2.0 * (s1[u][:, None, :] * s1[v][None, :, :] + s0[u][:, None, :] * s0[v][None, :, :])
                 + s1[u][:, None, :] * s0[v][None, :, :] + s0[u][:, None, :] * s1[v][None, :, :])  # (7b, 7c, n)
        pref = -(1.0 / 6.0) * (g.h[comp] / g.dt) * charge / g.V              # (n,)
        val = pref[None, None, None, :] * dF[comp][:, None, None, :] * brace[None, :, :, :]  # (a, b, c, n)
        ijk = [None, None, None]
        ijk[comp] = nodes[comp][:, None, None, :]
        ijk[u] = nodes[u][None, :, None, :]
        ijk[v] = nodes[v][None, None, :, :]
        idx = _flat(g, ijk[0], ijk[1], ijk[2]).expand_as(val)
        J.append(torch.zeros(nc, dtype=DT).index_add(0, idx.reshape(-1), val.reshape(-1)))
    return torch.stack(J).reshape(3, g.nz, g.ny, g.nx)


@dataclass
class Species:
    x: torch.Tensor        # (3, n) cell units
    w: torch.Tensor        # (3, n) momentum over mass at n - 1/2
    weight: torch.Tensor   # (n,)
    q: float = -1.0
    m: float = 1.0


def step(g: Grid, E, B, species, bext):
    """One Appendix step; returns E^{n+1}, B^{n+1/2} and the advanced species."""
    Bh = half_b(g, E, B)
    J = torch.zeros((3, g.nz, g.ny, g.nx), dtype=DT)
    out = []
    n = torch.tensor(g.n, dtype=DT)[:, None]
    for s in species:
        Ep, Bp = gather(g, E, Bh, s.x, bext)
        w = push(s.q / s.m, g.dt, g.c, Ep, Bp, s.w)
        x1 = s.x + displacement(g, w)
        J = J + deposit(g, s.x, x1, s.q * s.weight)
        out.append(Species(torch.remainder(x1, n), w, s.weight, s.q, s.m))
    B2 = half_b(g, E, Bh)
    return update_e(g, E, B2, J), B2, out


def field_energy(g: Grid, E, B):
    """V/(8 pi) sum E^2 + (B^n)^2, B^n = B^{n-1/2} advanced a half step."""
    Bn = half_b(g, E, B)
    return g.V / (8.0 * math.pi) * ((E * E).sum() + (Bn * Bn).sum())


def run(g: Grid, E, B, species, bext, nsteps):
    for _ in range(nsteps):
        E, B, species = step(g, E, B, species, bext)
    return E, B, species


def loss_and_grad(g: Grid, x, w, weight, q, m, bext, nsteps, E=None, B=None):
    """Final field energy after nsteps from E = B = 0 (or the given fields) and
    its gradients with respect to the initial momenta w (3, n), the external
    uniform field bext (3,) and the initial positions x (3, n, cell units):
    returns (L, dL/dw, dL/dbext, dL/dx)."""
    shape = (3, g.nz, g.ny, g.nx)
    E = torch.zeros(shape, dtype=DT) if E is None else torch.as_tensor(E, dtype=DT)
    B = torch.zeros(shape, dtype=DT) if B is None else torch.as_tensor(B, dtype=DT)
    w0 = torch.tensor(w, dtype=DT, requires_grad=True)
    b0 = torch.tensor(bext, dtype=DT, requires_grad=True)
    x0 = torch.tensor(x, dtype=DT, requires_grad=True)
    sp = [Species(x0, w0, torch.tensor(weight, dtype=DT), q, m)]
    E, B, _ = run(g, E, B, sp, b0, nsteps)
    L = field_energy(g, E, B)
    L.backward()
    return float(L.detach()), w0.grad.numpy(), b0.grad.numpy(), x0.grad.numpy()


def field_energy_grad_fields(g: Grid, E, B):
    """dL/dE and dL/dB^{n-1/2} of L = field_energy(E, B), by autograd."""
    E = torch.tensor(np.asarray(E), dtype=DT, requires_grad=True)
    B = torch.tensor(np.asarray(B), dtype=DT, requires_grad=True)
    field_energy(g, E, B).backward()
    return E.grad.numpy(), B.grad.numpy()


def step_vjp(g: Grid, E, B, x, w, weight, q, m, bext, lamE, lamB, lamx, lamw):
    """One step's vector-Jacobian product: given the adjoints (lamE, lamB,
    lamx, lamw) of the state after a step taken from (E, B, x, w) with one
    species, return those of the state before it and dL/dbext:
    (lamE, lamB, lamx, lamw, lambext)."""
    t = lambda a: torch.tensor(np.asarray(a), dtype=DT, requires_grad=True)
    E, B, x0, w0, b0 = t(E), t(B), t(x), t(w), t(bext)
    E1, B1, sp = step(g, E, B, [Species(x0, w0, torch.tensor(weight, dtype=DT), q, m)], b0)
    c = lambda a: torch.tensor(np.asarray(a), dtype=DT)
    L = ((E1 * c(lamE)).sum() + (B1 * c(lamB)).sum() + (sp[0].x * c(lamx)).sum()
         + (sp[0].w * c(lamw)).sum())
    L.backward()
    return E.grad.numpy(), B.grad.numpy(), x0.grad.numpy(), w0.grad.numpy(), b0.grad.numpy()


def loss_and_grad_species(g: Grid, species, bext, nsteps):
    """loss_and_grad for several mobile species: species is a list of
    (x, w, weight, q, m); returns (L, [(dL/dw, dL/dx) per species], dL/dbext)."""
    shape = (3, g.nz, g.ny, g.nx)
    E = torch.zeros(shape, dtype=DT)
    B = torch.zeros(shape, dtype=DT)
    b0 = torch.tensor(bext, dtype=DT, requires_grad=True)
    leaves, sp = [], []
    for x, w, weight, q, m in species:
        x0 = torch.tensor(x, dtype=DT, requires_grad=True)
        w0 = torch.tensor(w, dtype=DT, requires_grad=True)
        leaves.append((w0, x0))
        sp.append(Species(x0, w0, torch.tensor(weight, dtype=DT), q, m))
    E, B, _ = run(g, E, B, sp, b0, nsteps)
    L = field_energy(g, E, B)
    L.backward()
    return float(L.detach()), [(w0.grad.numpy(), x0.grad.numpy()) for w0, x0 in leaves], b0.grad.numpy()
