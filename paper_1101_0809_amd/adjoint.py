"""Gradients through the particle step: reverse sweep over the library's
hand-written adjoint kernels (include/pic.h, pic_adjoint_*).

The loss is the field energy V/(8 pi) sum E^2 + (B^n)^2 after a number of
steps (the energy diagnostic of Section 4.1).  Each reverse step reads the
state its forward step started from, kept as a record (pic_adjoint_record:
fields and particles, about 56 bytes per 2D particle).  With HBM to spare the
forward pass records every step (the tape) and the reverse pass reads it
back: one forward and one reverse step per step.  When the tape does not fit
the memory budget, the forward pass keeps a full state copy every ``every``
steps and the reverse pass re-runs each segment from its copy, recording the
segment's steps only while it walks back through them (one more forward step
per step, nsteps/every copies plus one segment of records).

Every step of the forward and of the reverse pass runs in the library's HIP
kernels; this module only orders the calls and holds the copies.
"""
from __future__ import annotations

import torch

from .sim import Sim


def _tape(sim: Sim, nsteps: int) -> torch.Tensor:
    rb = sim.adjoint_record_bytes()
    return torch.empty((nsteps, rb), dtype=torch.uint8, device=sim.device)


def _plan(sim: Sim, nsteps: int, every, budget_bytes) -> int:
    """Segment length: nsteps (a full tape) when every is None and the tape
    fits the budget (default half the free device memory), else every (20 if
    None)."""
    if every is not None:
        if every < 1:
            raise ValueError("every must be >= 1")
        return min(every, max(1, nsteps))
    if budget_bytes is None:
        budget_bytes = torch.cuda.mem_get_info(sim.device)[0] // 2
    if nsteps * sim.adjoint_record_bytes() <= budget_bytes:
        return max(1, nsteps)
    return 20


def _forward(sim: Sim, nsteps: int, seg: int):
    """Step the context nsteps times from its current state.  Returns the
    checkpoints [(length, state copy)] and, for a single segment, its tape."""
    if seg >= nsteps:
        tape = _tape(sim, max(1, nsteps))
        for i in range(nsteps):
            sim.adjoint_record(tape[i])
            sim.step(1)
        return [], tape
    ckpt = []
    done = 0
    while done < nsteps:
        k = min(seg, nsteps - done)
        ckpt.append((k, sim.snapshot()))
        sim.step(k)
        done += k
    return ckpt, None


def _field_energy(sim: Sim) -> float:
    d = sim.diagnostics()
    return d["field_e"] + d["field_b"]


def _reverse(sim: Sim, nsteps: int, ckpt: list, tape, lam_fields: torch.Tensor):
    """Walk back from the adjoint lam_fields of the final fields; return
    (lam_x, lam_w, lam_bext) of the state the forward pass started from
    (particle arrays per species, id order, None for immobile ones)."""
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
    if tape is not None:
        for i in reversed(range(nsteps)):
            sim.adjoint_step_record(tape[i], lam_fields, lam_x, lam_w, lam_b)
        return lam_x, lam_w, lam_b
    seg_tape = _tape(sim, max(k for k, _ in ckpt))
    for k, snap in reversed(ckpt):
        sim.restore(snap)
        for j in range(k):
            sim.adjoint_record(seg_tape[j])
            if j + 1 < k:
                sim.step(1)
        for j in reversed(range(k)):
            sim.adjoint_step_record(seg_tape[j], lam_fields, lam_x, lam_w, lam_b)
    return lam_x, lam_w, lam_b


def field_energy_grad(sim: Sim, nsteps: int, every: int = None, budget_bytes: int = None):
    """Advance ``sim`` by nsteps and return the final field energy L with its
    derivatives with respect to the state the context held on entry:
    (L, lam_x, lam_w, lam_bext), lam_x[s] and lam_w[s] of shape (3, n) in
    particle-id order (dL/dx in cell units, dL/dw), lam_bext = dL/dB_ext.
    every: checkpoint spacing; None records every step when the tape fits
    budget_bytes (default half the free device memory).  On return the
    context holds the state after the nsteps (as after sim.step(nsteps))."""
    seg = _plan(sim, nsteps, every, budget_bytes)
    ckpt, tape = _forward(sim, nsteps, seg)
    final = sim.snapshot() if tape is None else None
    L = _field_energy(sim)
    lam_f = torch.empty(6 * sim.ncell, dtype=torch.float64, device=sim.device)
    sim.adjoint_seed_field_energy(lam_f)
    gx, gw, gb = _reverse(sim, nsteps, ckpt, tape, lam_f)
    if final is not None:
        sim.restore(final)
    return L, gx, gw, gb


class _FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, w0, weight, bext, grid, q, m, nsteps, every):
        sim = Sim(**dict(grid, bext=tuple(float(v) for v in bext.detach().cpu())))
        sim.add_species(q, m, capacity=weight.numel())
        sim.load(0, x0.detach(), w0.detach(), weight.detach())
        ckpt, tape = _forward(sim, nsteps, _plan(sim, nsteps, every, None))
        L = _field_energy(sim)
        ctx.sim, ctx.ckpt, ctx.tape, ctx.nsteps = sim, ckpt, tape, nsteps
        ctx.devices = (x0.device, w0.device, bext.device)
        return torch.tensor(L, dtype=torch.float64, device=x0.device)

    @staticmethod
    def backward(ctx, grad_L):
        sim = ctx.sim
        lam_f = torch.empty(6 * sim.ncell, dtype=torch.float64, device=sim.device)
        sim.adjoint_seed_field_energy(lam_f)
        gx, gw, gb = _reverse(sim, ctx.nsteps, ctx.ckpt, ctx.tape, lam_f)
        ctx.sim = ctx.ckpt = ctx.tape = None
        sim.close()
        s = grad_L.to(sim.device, torch.float64)
        dx, dw, db = ctx.devices
        return ((gx[0] * s).to(dx), (gw[0] * s).to(dw), None, (gb * s).to(db),
                None, None, None, None, None)


def field_energy(x0: torch.Tensor, w0: torch.Tensor, weight: torch.Tensor, bext: torch.Tensor,
                 grid: dict, nsteps: int, q: float = -1.0, m: float = 1.0,
                 every: int = None) -> torch.Tensor:
    """Field energy after nsteps of one mobile species started from positions
    x0 (3, n, cell units), momenta w0 (3, n) and weights (n,) in a fresh
    context built from ``grid`` (keyword arguments of Sim, FP64, no plane-wave
    source) with uniform external field bext (3,).  Differentiable with
    respect to x0, w0 and bext (not weight) through the library's adjoint
    kernels; the forward pass keeps its tape (or, with ``every``, a state copy
    every ``every`` steps) until backward runs."""
    return _FieldEnergy.apply(x0, w0, weight, bext, grid, q, m, nsteps, every)
