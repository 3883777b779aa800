"""Gradients through the particle step: checkpointed reverse sweep over the
library's hand-written adjoint kernels (include/pic.h, pic_adjoint_*).

The loss is the field energy V/(8 pi) sum E^2 + (B^n)^2 after a number of
steps (the energy diagnostic of Section 4.1).  The reverse sweep needs, for
every step, the state it was taken from.  Storing all of them costs a full
state copy per step, so the forward pass keeps one copy every ``every``
steps and the reverse pass re-runs each segment from its copy, keeping the
segment's per-step states only while it walks back through them: about
nsteps/every + every state copies and one extra forward step per step.

Every step of the forward and of the reverse pass runs in the library's HIP
kernels; this module only orders the calls and holds the copies.
"""
from __future__ import annotations

import torch

from .sim import Sim


def _forward(sim: Sim, nsteps: int, every: int) -> list:
    """Step the context nsteps times from its current state; return the list
    of (start step, state copy) checkpoints."""
    if every < 1:
        raise ValueError("every must be >= 1")
    ckpt = []
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        ckpt.append((k, sim.snapshot()))
        sim.step(k)
        done += k
    return ckpt


def _field_energy(sim: Sim) -> float:
    d = sim.diagnostics()
    return d["field_e"] + d["field_b"]


def _reverse(sim: Sim, ckpt: list, lam_fields: torch.Tensor):
    """Walk the checkpoints backwards from the adjoint lam_fields of the final
    fields; return (lam_x, lam_w, lam_bext) of the state the first checkpoint
    holds (particle arrays per species, id order, None for immobile ones)."""
    dev = sim.device
    lam_x, lam_w = [], []
    for i, s in enumerate(sim.species):
        if s.mobile:
            n = sim.count(i)
            lam_x.append(torch.zeros((3, n), dtype=torch.float64, device=dev))
            lam_w.append(torch.zeros((3, n), dtype=torch.float64, device=dev))
        else:
            lam_x.append(None)
            lam_w.append(None)
    lam_b = torch.zeros(3, dtype=torch.float64, device=dev)
    for k, snap in reversed(ckpt):
        sim.restore(snap)
        states = []
        for j in range(k):
            states.append(sim.snapshot())
            if j + 1 < k:
                sim.step(1)
        for st in reversed(states):
            sim.restore(st)
            sim.adjoint_step(lam_fields, lam_x, lam_w, lam_b)
        del states
    return lam_x, lam_w, lam_b


def field_energy_grad(sim: Sim, nsteps: int, every: int = 20):
    """Advance ``sim`` by nsteps and return the final field energy L with its
    derivatives with respect to the state the context held on entry:
    (L, lam_x, lam_w, lam_bext), lam_x[s] and lam_w[s] of shape (3, n) in
    particle-id order (dL/dx in cell units, dL/dw), lam_bext = dL/dB_ext.
    On return the context holds the state after the nsteps (as after
    sim.step(nsteps))."""
    ckpt = _forward(sim, nsteps, every)
    final = sim.snapshot()
    L = _field_energy(sim)
    lam_f = torch.empty(6 * sim.ncell, dtype=torch.float64, device=sim.device)
    sim.adjoint_seed_field_energy(lam_f)
    gx, gw, gb = _reverse(sim, ckpt, lam_f)
    sim.restore(final)
    return L, gx, gw, gb


class _FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, w0, weight, bext, grid, q, m, nsteps, every):
        sim = Sim(**dict(grid, bext=tuple(float(v) for v in bext.detach().cpu())))
        sim.add_species(q, m, capacity=weight.numel())
        sim.load(0, x0.detach(), w0.detach(), weight.detach())
        ckpt = _forward(sim, nsteps, every)
        L = _field_energy(sim)
        ctx.sim, ctx.ckpt = sim, ckpt
        ctx.devices = (x0.device, w0.device, bext.device)
        return torch.tensor(L, dtype=torch.float64, device=x0.device)

    @staticmethod
    def backward(ctx, grad_L):
        sim, ckpt = ctx.sim, ctx.ckpt
        lam_f = torch.empty(6 * sim.ncell, dtype=torch.float64, device=sim.device)
        sim.adjoint_seed_field_energy(lam_f)
        gx, gw, gb = _reverse(sim, ckpt, lam_f)
        ctx.sim = ctx.ckpt = None
        sim.close()
        s = grad_L.to(sim.device, torch.float64)
        dx, dw, db = ctx.devices
        return ((gx[0] * s).to(dx), (gw[0] * s).to(dw), None, (gb * s).to(db),
                None, None, None, None, None)


def field_energy(x0: torch.Tensor, w0: torch.Tensor, weight: torch.Tensor, bext: torch.Tensor,
                 grid: dict, nsteps: int, q: float = -1.0, m: float = 1.0,
                 every: int = 20) -> torch.Tensor:
    """Field energy after nsteps of one mobile species started from positions
    x0 (3, n, cell units), momenta w0 (3, n) and weights (n,) in a fresh
    context built from ``grid`` (keyword arguments of Sim, FP64, no plane-wave
    source) with uniform external field bext (3,).  Differentiable with
    respect to x0, w0 and bext (not weight) through the library's adjoint
    kernels; the forward pass keeps a state copy every ``every`` steps until
    backward runs."""
    return _FieldEnergy.apply(x0, w0, weight, bext, grid, q, m, nsteps, every)
