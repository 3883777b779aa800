"""Throughput benchmark: particle-steps per second of the charge-conserving PIC
step on one MI355X, FP32-compensated and FP64, with the roofline position of
the particle kernel and the FP64 CPU oracle timed on the host beside it.

Workload (default): the largest single-GPU one, 3D3V on 256^3 periodic cells
with 32 electrons and 32 mobile ions (mass ratio 100) per cell, 1,073,741,824
particles, bi-Maxwellian electrons w_th = (0.3, 0.05, 0.05) c, ions
w_th = 0.005 c, dt = 0.45 dx/c, particles re-sorted by cell every 20 steps;
drawn on the GPU from seeded generators.  Its stated mode, FP32-compensated,
leads the line; FP64 runs beside it on the same workload, and the FP32c error
against FP64 after the same steps is reported.  One "step" is the whole step:
both B half steps, the particle kernel of each species (gather, push,
deposit) and the E update, plus the periodic sort when due.  Inputs are
resident on the GPU before the timed region starts.  The K timed steps carry
no per-phase events; a second pass of one sort period with HIP events around
each phase gives the per-kernel durations of the roofline and the phase
breakdown.

    python bench.py [--gpus 1] [--steps 40] [--warmup 5]

prints one JSON line.  Other measurements, each printing its own line:
--workload NAME (another workload of picgen.WORKLOADS), --order 2 (the
alternating order 2 1/2), --interp conventional (the uniform-order gather of
Eq. wrong1), --adjoint (gradient time over forward time of the 2D3V
differentiable workload, or of --workload), --copy-probe (a plain device copy
for scaling rocprofv3 byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
DEFAULT_WORKLOAD = "3d_256cube_weibel"
# the precision a workload is stated in leads its line; the other runs beside it
HEADLINE_PRECISION = {"3d_256cube_weibel": "fp32c"}


def particle_bytes(precision: str, dims: int) -> int:
    """Algorithmic HBM bytes per particle per step of the particle kernel:
    particle state read once and written once."""
    if precision == "fp64":
        # read x (8*dims) + w 24 + weight 8; write x (8*dims) + w 24
        return 2 * 8 * dims + 2 * 24 + 8
    # read cell 4 + offsets (4*dims) + w 12 + weight 4; write cell 4 + offsets + w 12
    return 2 * (4 + 4 * dims + 12) + 4


def grid_bytes_particle_kernel() -> int:
    """Per cell per launch: E and B^n read once (6 FP64), J written once (3 FP64)."""
    return 9 * 8


DEVICE_DRAW = 1 << 26  # species at least this large are drawn on the GPU (picgen.device_chunks)


def load_workload(sim, wl):
    """Electrons, plus ions co-located with them: a second mobile species when
    the workload's ions move, else the immobile background.  Large species
    are drawn on the GPU in seeded chunks, the others on the host.  Returns
    the indices of the mobile species."""
    import picgen

    n = wl.n_electrons
    se = sim.add_species(-1.0, 1.0, n)
    si = sim.add_species(1.0, wl.ion_mass, n if wl.ions_mobile else 0, mobile=wl.ions_mobile)
    if n >= DEVICE_DRAW:
        for sp, ions in ((se, False), (si, True)):
            for x, w, wt in picgen.device_chunks(wl, sim.device, ions=ions):
                sim.load(sp, x, w, wt)
                del x, w, wt
    else:
        e = picgen.electrons(wl)
        ion = picgen.ions_like(wl, e)
        sim.load(se, e.x, e.w, e.weight)
        sim.load(si, ion.x, ion.w, ion.weight)
    return [se, si] if wl.ions_mobile else [se]


def sampled_state(sim, species, per_species: int = 16384):
    """E, B (host copies) and, per mobile species, about per_species particles
    (those whose id is a multiple of a stride), in id order: (x, w) host
    arrays.  For comparing two runs of one workload."""
    import ctypes

    import torch

    F = sim.fields_numpy()[:6].copy()
    parts = []
    for sp in species:
        n = sim.count(sp)
        stride = max(1, n // per_species)
        x = torch.empty((3, n), dtype=torch.float64, device=sim.device)
        w = torch.empty((3, n), dtype=torch.float64, device=sim.device)
        pid = torch.empty(n, dtype=torch.int64, device=sim.device)
        sim._check(sim.lib.pic_get_particles(sim.ctx, sp, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(w.data_ptr()), None,
                                              ctypes.c_void_p(pid.data_ptr()),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        idx = torch.nonzero(pid % stride == 0).flatten()
        order = torch.argsort(pid[idx])
        idx = idx[order]
        parts.append((x[:, idx].cpu().numpy(), w[:, idx].cpu().numpy()))
        del x, w, pid, idx, order
        torch.cuda.empty_cache()
    return F, parts


def run_gpu(wl, precision: str, steps: int, warmup: int, order: int = 1, interp: str = "alternating",
            sample: bool = False, xbc: str = "periodic"):
    import torch

    from paper_1101_0809_amd import Sim

    sim = Sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision=precision,
              sort_every=wl.sort_every, bext=wl.bext, order=order, interp=interp, source=wl.source,
              xbc=xbc)
    species = load_workload(sim, wl)
    torch.cuda.empty_cache()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    # timed pass: whole steps only (per-phase events would add their own gaps)
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    # a second pass with HIP events around every phase, on the stream the
    # kernels run on: per-kernel durations for the roofline.  It spans one
    # sort period (at least 20 steps), so the sort share is the run's.
    tsteps = max(min(steps, max(20, wl.sort_every)), 1)
    sim.timing_start(tsteps)
    sim.step(tsteps)
    torch.cuda.synchronize()
    phases = sim.timing_stop()
    fallback = sim.fallback_fraction()
    migrant = sim.migrant_fraction()
    d = sim.diagnostics()
    counts = [sim.count(s) for s in species]
    snap = sampled_state(sim, species) if sample else None
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"n": sum(counts), "counts": counts, "ms_per_step": total_ms / steps, "phases": phases,
            "diag": d, "fallback": fallback, "migrant": migrant, "sample": snap, "steps_total": warmup + steps + tsteps}


def precision_error(r32, r64):
    """FP32c against FP64 on the same workload after the same steps: relative
    2-norm error of E and of B, and the largest momentum and position error
    of the sampled particles (matched by id)."""
    import numpy as np

    F32, P32 = r32["sample"]
    F64, P64 = r64["sample"]
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    out = {"E_rel_l2": rel(F32[:3], F64[:3]), "B_rel_l2": rel(F32[3:6], F64[3:6])}
    werr, xerr, m = 0.0, 0.0, 0
    for (x32, w32), (x64, w64) in zip(P32, P64):
        if w64.size == 0:
            continue
        werr = max(werr, float(np.max(np.abs(w32 - w64)) / np.max(np.abs(w64))))
        dx = x32 - x64
        for a, n in enumerate(F64.shape[1:][::-1]):
            dx[a] -= n * np.round(dx[a] / n)
        xerr = max(xerr, float(np.max(np.abs(dx))))
        m += w64.shape[1]
    d32, d64 = r32["diag"], r64["diag"]
    out.update({"w_rel_max": werr, "x_abs_max_cells": xerr, "sampled_particles": m,
                "kinetic_rel": abs(d32["kinetic"] - d64["kinetic"]) / abs(d64["kinetic"]),
                "field_energy_rel": abs(d32["field_e"] + d32["field_b"] - d64["field_e"] - d64["field_b"])
                / abs(d64["field_e"] + d64["field_b"]),
                "after_steps": r64["steps_total"],
                "sample": "fields: all cells; particles: about 16384 per species (ids on a fixed stride)"})
    return out


def adjoint_bytes(dims: int):
    """Algorithmic HBM bytes of one reverse step (FP64): per particle, the state
    read once (x 8*dims, w 24, weight 8, id 8) and its adjoint read and written
    once (dL/dx 8*dims read, 24 written; dL/dw 24 + 24); per cell, the grid
    planes each of the five kernels must touch: B^n from E, B (6 read, 3
    written), lambda_J and lambda_B from lambda_E' (3 read, 3 + 3 read-write
    for lambda_B, 3 written), two curl passes (3 read, 3 read-write each), the
    particle pass (E, B^n, lambda_J read; lambda_E, lambda_B read-write)."""
    per_particle = 8 * dims + 24 + 8 + 8 + (8 * dims + 24) + (24 + 24)
    per_cell = 8 * (9 + 12 + 2 * 9 + 21)
    return per_particle, per_cell


def run_adjoint(wl, every: int):
    """Field-energy gradient of wl (FP64): forward time of wl.steps steps, the
    whole gradient (forward pass with its records or checkpoints, reverse
    steps), one reverse step and one record on their own."""
    import torch

    import picgen
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd.adjoint import field_energy_grad

    e = picgen.electrons(wl)
    sim = Sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision="fp64",
              sort_every=wl.sort_every, bext=wl.bext)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    n = e.n
    del e
    init = sim.snapshot()
    field_energy_grad(sim, 4, every=2)       # warm-up of every kernel and copy
    sim.restore(init)
    field_energy_grad(sim, 2)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()

    sim.restore(init)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    sim.step(wl.steps)
    b.record(stream)
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b)

    def timed_grad(ev_every):
        sim.restore(init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = field_energy_grad(sim, wl.steps, every=ev_every)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, out

    grad_ms, (L, gx, gw, gb) = timed_grad(every)
    # the other storage mode beside it: the tape when checkpoints lead, and
    # checkpoints every 20 steps when the tape leads
    other_every = None if every else 20
    other_ms, (L2, _, _, gb2) = timed_grad(other_every)

    # one reverse step from a record of a sorted state (as every step after
    # the first; particle adjoints in storage order, as in the sweep),
    # repeated, and the record copy alone
    sim.restore(init)
    sim.step(1)
    rec = torch.empty(sim.adjoint_record_bytes(), dtype=torch.uint8, device=sim.device)
    sim.adjoint_record(rec)
    lam_f = torch.zeros(6 * sim.ncell, dtype=torch.float64, device=sim.device)
    sim.adjoint_seed_field_energy(lam_f)
    lx = [torch.zeros((3, n), dtype=torch.float64, device=sim.device)]
    lw = [torch.zeros((3, n), dtype=torch.float64, device=sim.device)]
    lb = torch.zeros(3, dtype=torch.float64, device=sim.device)
    reps = 20
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        sim.adjoint_step_record(rec, lam_f, lx, lw, lb, ordered=True)
    b.record(stream)
    torch.cuda.synchronize()
    adj_ms = a.elapsed_time(b) / reps
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        sim.adjoint_record(rec)
    b.record(stream)
    torch.cuda.synchronize()
    copy_ms = a.elapsed_time(b) / reps
    record_bytes = rec.numel()
    sim.close()
    pp, pc = adjoint_bytes(wl.dims)
    nbytes = n * pp + wl.ncell * pc
    achieved = nbytes / (adj_ms * 1e-3) / 1e9
    return {"n": n, "forward_ms": fwd_ms, "grad_ms": grad_ms, "adjoint_step_ms": adj_ms,
            "record_ms": copy_ms, "record_bytes": record_bytes, "loss": L,
            "dL_dbext": gb.cpu().tolist(),
            "other": {"checkpoint_every": other_every or "none (tape of every step)",
                      "grad_ms": other_ms, "x_forward": other_ms / fwd_ms,
                      "dL_dbext_rel_diff": float((gb2 - gb).abs().max() / gb.abs().max().clamp_min(1e-300))},
            "bytes_per_reverse_step": nbytes, "achieved_gbs": achieved}


def measured_traffic(precision: str, workload: str):
    """HBM bytes per particle-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or
    None if there is none or the kernel source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_particle_step_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- traffic-json (\{.*\}) -->", open(path).read())
    if not m:
        return None
    info = json.loads(m.group(1))
    # the step kernels' sources: the kernel file and the two headers it builds on
    h = hashlib.sha256()
    for name in ("particles.hip", "pic_math.h", "pic_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1101_0809_amd", "csrc", name), "rb").read())
    digest = h.hexdigest()[:16]
    if info.get("source_sha256_16") != digest:
        return None
    return info["traffic"].get(precision)


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM bandwidth: a plain device-to-device copy of 1 GiB (larger
    than the 256 MB Infinity Cache), read + write bytes over the mean time."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2 * nbytes / sec / 1e9


def roofline(res, precision, wl, copy_gbs=None, order=1, interp="alternating"):
    """Position of the particle kernel against the HBM roofline.  One launch
    advances one mobile species: its particles' state is read and written
    once and the grid's E, B^n read and J written once.  achieved = those
    algorithmic bytes per launch over the launch's average duration (HIP
    events on the kernels' stream)."""
    nlaunch = len(res["counts"])
    per_launch_ms = res["phases"]["particles"] / max(1, res["phases"]["steps"]) / nlaunch
    bytes_launch = (res["n"] * particle_bytes(precision, wl.dims)
                    + nlaunch * wl.ncell * grid_bytes_particle_kernel()) / nlaunch
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    kernel = "k_particle_step3" if wl.dims == 3 else "k_particle_step"
    traffic = measured_traffic(precision, wl.name)
    if order == 2:
        kernel = "k_push_o2_3d + k_deposit_o2_3d" if wl.dims == 3 else "k_step_o2<2>"
        traffic = None
    elif interp == "conventional":
        kernel = "k_push_conv3 + k_deposit_conv3" if wl.dims == 3 else "k_step_conv2"
        traffic = None
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_launch": int(bytes_launch),
            "bytes_per_particle_step": round(bytes_launch * nlaunch / res["n"], 2),
            "launches_per_step": nlaunch,
            "avg_launch_ms": round(per_launch_ms, 5),
            "copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
            "frac_of_copy": None if copy_gbs is None else round(achieved / copy_gbs, 4)}


def _oracle_state(wl, e, ion, order=1, interp="alternating", xbc=0):
    import oracle

    sp = [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m)] if e is not None else []
    if ion is not None:
        sp.append(oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=wl.ions_mobile))
    return oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext, order=order,
                                    interp=1 if interp == "conventional" else 0, source=wl.source,
                                    xbc=xbc), sp)


def cpu_baseline(wl, min_seconds: float = 10.0, max_steps: int = 12, order: int = 1,
                 interp: str = "alternating", full_limit: int = 1 << 22, sample_n: int = 1 << 20,
                 all_cores: bool = True, xbc: int = 0):
    """The FP64 oracle as it stands, serial, on the host.  A workload of at
    most full_limit mobile particles runs whole steps (all particles, full
    grid), as many as take min_seconds (at most max_steps).  A larger one is
    sampled: one step of the full grid without particles (the field updates)
    and one step of the full grid with sample_n electrons (and as many ions
    when they move) drawn from the workload's distributions; the per-particle
    time of the second, with the grid time of the first, gives the rate of a
    step of the whole workload; with all_cores, the sampled form also runs on
    every host core at once (cpu_all_cores)."""
    import picgen

    host = (f"host {platform.processor() or platform.machine()} "
            f"({os.cpu_count()} logical CPUs, 1 used)")
    if wl.n_particles <= full_limit:
        e = picgen.electrons(wl)
        ion = picgen.ions_like(wl, e)
        st = _oracle_state(wl, e, ion, order, interp, xbc)
        t0 = time.perf_counter()
        sample_steps = 0
        while sample_steps < max_steps and (sample_steps == 0 or time.perf_counter() - t0 < min_seconds):
            st.step(1)
            sample_steps += 1
        dt = time.perf_counter() - t0
        return {"value": round(wl.n_particles * sample_steps / dt, 1), "unit": "particle-steps/s",
                "cores": 1, "kind": "oracle",
                "sample": f"{sample_steps} full step(s) of the same workload ({wl.n_particles} particles, "
                          f"order {order} 1/2, {interp} interpolation, {wl.nx}x{wl.ny}x{wl.nz} grid), "
                          f"serial C oracle, {dt:.1f} s, {host}"}
    grid_only = _oracle_state(wl, None, None, order, interp, xbc)
    t0 = time.perf_counter()
    grid_only.step(1)
    t_grid = time.perf_counter() - t0
    del grid_only
    t_step, ns = _oracle_sample_step(wl, sample_n, order, interp, xbc)
    t_pp = max(t_step - t_grid, 1e-12) / ns
    t_full = t_grid + wl.n_particles * t_pp
    out = {"value": round(wl.n_particles / t_full, 1), "unit": "particle-steps/s", "cores": 1,
           "kind": "oracle",
           "sample": f"full {wl.nx}x{wl.ny}x{wl.nz} grid: one oracle step without particles "
                     f"({t_grid:.2f} s, the field updates) and one with {ns} particles drawn from the "
                     f"workload's distributions ({t_step:.2f} s); rate of the whole workload "
                     f"({wl.n_particles} particles) = N / (grid time + N x per-particle time), "
                     f"serial C oracle, order {order} 1/2, {interp} interpolation, {host}"}
    if all_cores:
        out["all_cores"] = cpu_all_cores(wl, t_grid, sample_n, order, interp, xbc=xbc)
    return out


def _oracle_sample_step(wl, sample_n, order, interp, xbc=0):
    """One oracle step of the full grid with sample_n electrons (and as many
    ions when they move) drawn from the workload's distributions: (seconds,
    particles stepped)."""
    import picgen

    small = wl.scaled(ppc=1)
    e = picgen.electrons(small, n=sample_n)
    e.weight[:] = wl.weight
    ion = picgen.ions_like(wl, e)
    st = _oracle_state(wl, e, ion, order, interp, xbc)
    ns = sample_n * (2 if wl.ions_mobile else 1)
    t0 = time.perf_counter()
    st.step(1)
    return time.perf_counter() - t0, ns


def cpu_all_cores(wl, t_grid, sample_n, order, interp, procs=None, xbc=0):
    """The serial oracle on every host core at once: one child process per
    core (at most 16), each stepping its own sample as the serial leg does.
    The particles of a step are independent, so P copies stepping P samples
    side by side give the host's rate for the particle work; the field
    update (t_grid, serial) is added once.  Children are separate programs
    started after the parent has used the GPU, not forks of it."""
    import subprocess

    procs = procs or max(1, min(16, os.cpu_count() or 1))
    code = (f"import json, sys; sys.path.insert(0, {ROOT!r}); import bench, picgen; "
            f"wl = picgen.WORKLOADS[{wl.name!r}]; "
            f"t, ns = bench._oracle_sample_step(wl, {sample_n}, {order}, {interp!r}, {xbc}); "
            f"print(json.dumps({{'t': t, 'ns': ns}}))")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    t0 = time.perf_counter()
    ch = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                           env=env, text=True) for _ in range(procs)]
    res = []
    for c in ch:
        out, _ = c.communicate()
        if c.returncode != 0:
            raise RuntimeError(f"oracle child failed with status {c.returncode}")
        res.append(json.loads(out.strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    t_slow = max(r["t"] for r in res)   # every child's particle step overlaps the others'
    ns_all = sum(r["ns"] for r in res)
    t_pp = max(t_slow - t_grid, 1e-12) / ns_all
    t_full = t_grid + wl.n_particles * t_pp
    return {"value": round(wl.n_particles / t_full, 1), "unit": "particle-steps/s", "cores": procs,
            "kind": "oracle",
            "sample": f"{procs} copies of the serial C oracle side by side, one per core, each stepping "
                      f"its own {res[0]['ns']} particles on the full grid (slowest step {t_slow:.2f} s, "
                      f"{wall:.1f} s wall with set-up); per-particle time = slowest step / all particles, "
                      f"plus one serial field update"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None,
                    help=f"workload name (default {DEFAULT_WORKLOAD}; 2d3v_256sq_beams with --adjoint)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["both", "fp64", "fp32c"], default="both")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB (5 times), the reference "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the throughput line, time the checkpointed field-energy "
                         "gradient of the 2D3V 256x256 beams workload (FP64) against its forward "
                         "pass and print that as the one JSON line")
    ap.add_argument("--order", type=int, choices=[1, 2], default=1,
                    help="alternating form-factor order l_a = order + 1/2 (2: FP64 only)")
    ap.add_argument("--interp", choices=["alternating", "conventional"], default="alternating",
                    help="field interpolation: the alternating-order form factor, or the conventional "
                         "uniform order of Eq. wrong1 (the comparison of Section 5; FP64, order 1)")
    ap.add_argument("--xbc", choices=["periodic", "open"], default=None,
                    help="x boundary: periodic, or open (Mur walls, particles absorbed near them); "
                         "default: the workload's own (open for the 128^3 slab with the laser)")
    ap.add_argument("--every", type=int, default=None,
                    help="checkpoint spacing of --adjoint (default: 20 for the differentiable 2D3V "
                         "workload, its stated spacing; otherwise a tape of every step when it fits "
                         "in half the free device memory); the other mode is timed beside it")
    args = ap.parse_args(argv)
    if args.adjoint and args.gpus == 1:
        import picgen
        wl = picgen.WORKLOADS[args.workload or "2d3v_256sq_beams"]
        if args.every is None and wl.name == "2d3v_256sq_beams":
            args.every = 20   # the differentiable workload's stated checkpoint spacing
        r = run_adjoint(wl, args.every)
        fwd_step = r["forward_ms"] / wl.steps
        line = {
            "metric": "field-energy gradient time / forward time (adjoint, FP64)",
            "value": round(r["grad_ms"] / r["forward_ms"], 3),
            "unit": "x forward",
            "n_gpus": 1, "steps": wl.steps, "warmup": 4,
            "ms_per_step": round(r["grad_ms"] / wl.steps, 5),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "particles": r["n"],
                       "dt": wl.dt, "sort_every": wl.sort_every,
                       "checkpoint_every": args.every or "none (tape of every step)",
                       "bext": list(wl.bext), "parallelism": "none (1 GPU)"},
            "forward_ms_per_step": round(fwd_step, 5),
            "forward_particle_steps_per_s": round(r["n"] * 1e3 / fwd_step, 1),
            "reverse_step_ms": round(r["adjoint_step_ms"], 5),
            "reverse_step_x_forward_step": round(r["adjoint_step_ms"] / fwd_step, 3),
            "record_ms": round(r["record_ms"], 5), "record_bytes": r["record_bytes"],
            "roofline": {"bound": "hbm", "kernel": "reverse step (k_adj_* kernels)",
                         "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                         "traffic": None, "bytes_per_launch": r["bytes_per_reverse_step"],
                         "avg_launch_ms": round(r["adjoint_step_ms"], 5)},
            "loss": r["loss"], "dL_dbext": r["dL_dbext"],
            "other_mode": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r["other"].items()},
        }
        print(json.dumps(line), flush=True)
        return 0
    if args.copy_probe:
        import torch
        n = 256 * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                          "launches": 5}))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU "
                                   "decomposition is a design (see the design notes), "
                                   "rerun with --gpus 1"}))
        return 2

    import picgen
    wl = picgen.WORKLOADS[args.workload or DEFAULT_WORKLOAD]
    if args.xbc is None:
        args.xbc = wl.xbc
    head = HEADLINE_PRECISION.get(wl.name, "fp64")
    other = "fp64" if head == "fp32c" else "fp32c"
    precs = [head, other] if args.precision == "both" else [args.precision]
    if args.order == 2 or args.interp == "conventional":
        precs = ["fp64"]
    results = {}
    for p in precs:
        print(f"# {wl.name} {p}: loading {wl.n_particles} particles, {args.warmup} + {args.steps} steps",
              file=sys.stderr, flush=True)
        results[p] = run_gpu(wl, p, args.steps, args.warmup, args.order, args.interp,
                             sample=len(precs) == 2, xbc=args.xbc)
        r = results[p]
        print(f"# {p}: {r['ms_per_step']:.4f} ms/step, particle kernels "
              f"{r['phases']['particles'] / max(1, r['phases']['steps']):.4f} ms/step, "
              f"gauss_rel {r['diag']['gauss_rel']:.2e}, fallback {r['fallback']:.6f}, "
              f"migrants {r['migrant']:.6f}",
              file=sys.stderr, flush=True)
    copy_gbs = copy_bandwidth()
    main_p = precs[0]
    r = results[main_p]
    value = r["n"] * 1000.0 / r["ms_per_step"]
    line = {
        "metric": "particle-steps/sec on 1 MI355X (FP64 vs FP32-compensated) + % HBM roofline",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "particles": r["n"],
                   "particles_per_species": r["counts"], "ppc": wl.ppc,
                   "mobile_ions": wl.ions_mobile, "dt": wl.dt, "sort_every": wl.sort_every,
                   "precision": main_p, "order": f"{args.order} 1/2", "interp": args.interp,
                   "xbc": args.xbc,
                   "parallelism": "none (1 GPU)"},
        "roofline": roofline(r, main_p, wl, copy_gbs, args.order, args.interp),
        "phases_ms_per_step": {k: round(v / max(1, r["phases"]["steps"]), 5)
                               for k, v in r["phases"].items() if k != "steps"},
        "checks": {"gauss_rel": r["diag"]["gauss_rel"], "nonfinite": r["diag"]["nonfinite"],
                   "fallback_fraction": r["fallback"], "migrant_fraction": r["migrant"]},
    }
    if len(precs) == 2:
        ro = results[other]
        vo = ro["n"] * 1000.0 / ro["ms_per_step"]
        v64, v32 = (vo, value) if other == "fp64" else (value, vo)
        line[other] = {"value": round(vo, 1), "ms_per_step": round(ro["ms_per_step"], 5),
                       "roofline": roofline(ro, other, wl, copy_gbs),
                       "phases_ms_per_step": {k: round(v / max(1, ro["phases"]["steps"]), 5)
                                              for k, v in ro["phases"].items() if k != "steps"},
                       "gauss_rel": ro["diag"]["gauss_rel"], "fallback_fraction": ro["fallback"],
                       "migrant_fraction": ro["migrant"]}
        line["fp32c_speedup_vs_fp64"] = round(v32 / v64, 3)
        line["fp32c_error_vs_fp64"] = precision_error(results["fp32c"], results["fp64"])
    line["context"] = {"paper": "about 2.1e5 particles advanced per second of CPU time per processor "
                                "(FP64, order 1 1/2, 64^3 grid, 2 electrons per cell; Section 5); "
                                "another machine, not a target"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, order=args.order, interp=args.interp,
                                            xbc=1 if args.xbc == "open" else 0)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
