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


def _step_recorded(sim: Sim, record: torch.Tensor) -> bool:
    """Record the current state, take one step; return whether the step
    changed the storage order of the particles (it sorted)."""
    sim.adjoint_record(record)
    before = sim.host_state()
    unsorted = any(not before.sorted[i] for i, s in enumerate(sim.species) if s.mobile)
    sim.step(1)
    return unsorted or (sim.desc.sort_every > 0 and sim.host_state().since_sort == 0)


def _forward(sim: Sim, nsteps: int, seg: int):
    """Step the context nsteps times from its current state.  Returns the
    checkpoints [(length, state copy)] and, for a single segment, its tape
    with the steps that sorted."""
    # a species not yet sorted (just loaded) would be sorted by its first
    # step anyway; sorting it now only reorders storage, and lets the reverse
    # step of that first step use the tiled kernel
    hs = sim.host_state()
    if any(not hs.sorted[i] for i, s in enumerate(sim.species) if s.mobile):
        sim.sort()
        after = sim.host_state()
        after.since_sort = hs.since_sort  # keep the periodic sorts where they were
        sim.set_host_state(after)
    if seg >= nsteps:
        tape = _tape(sim, max(1, nsteps))
        sorted_at = [_step_recorded(sim, tape[i]) for i in range(nsteps)]
        return [], (tape, sorted_at)
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


class _ParticleAdjoint:
    """Particle adjoints of every species in one storage order, with a spare
    pair for out-of-place reordering."""

    def __init__(self, sim: Sim):
        self.sim = sim
        dev = sim.device
        mk = lambda i, s: (torch.zeros((3, sim.count(i)), dtype=torch.float64, device=dev)
                           if s.mobile else None)
        self.x = [mk(i, s) for i, s in enumerate(sim.species)]
        self.w = [mk(i, s) for i, s in enumerate(sim.species)]
        self.x2 = [None if t is None else torch.empty_like(t) for t in self.x]
        self.w2 = [None if t is None else torch.empty_like(t) for t in self.w]

    def reorder(self, src, dst):
        self.sim.adjoint_reorder(src, dst, self.x, self.w, self.x2, self.w2)
        self.x, self.x2 = self.x2, self.x
        self.w, self.w2 = self.w2, self.w


def _sweep(sim: Sim, records, sorted_at, lam_fields, pa: _ParticleAdjoint, lam_b):
    """Reverse steps over records[k-1] .. records[0]; the particle adjoints
    enter in the order of records[k-1] and leave in that of records[0]."""
    k = len(sorted_at)
    for j in reversed(range(k)):
        if j + 1 < k and sorted_at[j]:
            pa.reorder(records[j + 1], records[j])
        sim.adjoint_step_record(records[j], lam_fields, pa.x, pa.w, lam_b, ordered=True)


def _reverse(sim: Sim, nsteps: int, ckpt: list, tape, lam_fields: torch.Tensor):
    """Walk back from the adjoint lam_fields of the final fields; return
    (lam_x, lam_w, lam_bext) of the state the forward pass started from
    (particle arrays per species, id order, None for immobile ones)."""
    pa = _ParticleAdjoint(sim)
    lam_b = torch.zeros(3, dtype=torch.float64, device=sim.device)
    if tape is not None:
        records, sorted_at = tape
        # the adjoints start at zero: any order is the order of the last record
        _sweep(sim, records, sorted_at, lam_fields, pa, lam_b)
        if nsteps:
            pa.reorder(records[0], None)
        return pa.x, pa.w, lam_b
    seg_tape = _tape(sim, max(k for k, _ in ckpt))
    for k, snap in reversed(ckpt):
        sim.restore(snap)
        sorted_at = []
        for j in range(k):
            if j + 1 < k:
                sorted_at.append(_step_recorded(sim, seg_tape[j]))
            else:
                sim.adjoint_record(seg_tape[j])
                sorted_at.append(False)
        pa.reorder(None, seg_tape[k - 1])
        _sweep(sim, seg_tape, sorted_at, lam_fields, pa, lam_b)
        pa.reorder(seg_tape[0], None)
    return pa.x, pa.w, lam_b


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
