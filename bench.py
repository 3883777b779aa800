"""Throughput benchmark: particle-steps per second of the charge-conserving PIC
step on one MI355X, FP64 and FP32-compensated, with the roofline position of
the particle kernel and the FP64 CPU oracle timed on the host beside it.

Workload (default): 3D3V, 64^3 periodic cells, 8 electrons per cell
(2,097,152 electrons), Gaussian momenta w_th = 0.1 c, co-located immobile ions,
dt = 0.45 dx/c, particles re-sorted by cell every 10 steps.  One "step" is the
whole step: both B half steps, particle kernel (gather, push, deposit) and E
update, plus the periodic sort when due.  Inputs are resident on the GPU
before the timed region starts.  The K timed steps carry no per-phase events;
K further steps with HIP events around each phase give the per-kernel
durations of the roofline and the phase breakdown.

    python bench.py [--gpus 1] [--steps 50] [--warmup 10]

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


def run_gpu(wl, precision: str, steps: int, warmup: int, order: int = 1, interp: str = "alternating"):
    import numpy as np
    import torch

    import picgen
    from paper_1101_0809_amd import Sim

    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = Sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision=precision,
              sort_every=wl.sort_every, bext=wl.bext, order=order, interp=interp)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    del e, ion
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
    # second pass of as many steps with HIP events around every phase, on the
    # stream the kernels run on: per-kernel durations for the roofline
    sim.timing_start(steps)
    sim.step(steps)
    torch.cuda.synchronize()
    phases = sim.timing_stop()
    fallback = sim.fallback_fraction()
    d = sim.diagnostics()
    n = sim.count(s)
    sim.close()
    return {"n": n, "ms_per_step": total_ms / steps, "phases": phases, "diag": d,
            "fallback": fallback}


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

    sim.restore(init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, gx, gw, gb = field_energy_grad(sim, wl.steps, every=every)
    torch.cuda.synchronize()
    grad_ms = (time.perf_counter() - t0) * 1e3

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
            "bytes_per_reverse_step": nbytes, "achieved_gbs": achieved}


def measured_traffic(precision: str, workload: str):
    """HBM bytes per particle-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or
    None if there is none or the kernel source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_particle_step_{workload}.md")
    src = os.path.join(ROOT, "paper_1101_0809_amd", "csrc", "particles.hip")
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- traffic-json (\{.*\}) -->", open(path).read())
    if not m:
        return None
    info = json.loads(m.group(1))
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
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
    per_launch_ms = res["phases"]["particles"] / max(1, res["phases"]["steps"])
    bytes_launch = (res["n"] * particle_bytes(precision, wl.dims)
                    + wl.ncell * grid_bytes_particle_kernel())
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
            "traffic": traffic, "bytes_per_launch": bytes_launch,
            "avg_launch_ms": round(per_launch_ms, 5),
            "copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
            "frac_of_copy": None if copy_gbs is None else round(achieved / copy_gbs, 4)}


def cpu_baseline(wl, min_seconds: float = 10.0, max_steps: int = 12, order: int = 1,
                 interp: str = "alternating"):
    """The FP64 oracle as it stands, serial, on the host: whole steps of the
    full workload (all particles, full grid), as many as take min_seconds
    (at most max_steps)."""
    import oracle
    import picgen

    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext, order=order,
                                  interp=1 if interp == "conventional" else 0),
                      [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m),
                       oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False)])
    t0 = time.perf_counter()
    sample_steps = 0
    while sample_steps < max_steps and (sample_steps == 0 or time.perf_counter() - t0 < min_seconds):
        st.step(1)
        sample_steps += 1
    dt = time.perf_counter() - t0
    return {"value": round(e.n * sample_steps / dt, 1), "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_steps} full step(s) of the same workload ({e.n} particles, order {order} 1/2, "
                      f"{interp} interpolation, "
                      f"{wl.nx}x{wl.ny}x{wl.nz} grid), serial C oracle, {dt:.1f} s, "
                      f"host {platform.processor() or platform.machine()} "
                      f"({os.cpu_count()} logical CPUs, 1 used)"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=None,
                    help="workload name (default 3d_64cube_8ppc; 2d3v_256sq_beams with --adjoint)")
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
    ap.add_argument("--every", type=int, default=None,
                    help="checkpoint spacing of --adjoint (default: record every step when the "
                         "tape fits in half the free device memory)")
    args = ap.parse_args(argv)
    if args.adjoint and args.gpus == 1:
        import picgen
        wl = picgen.WORKLOADS[args.workload or "2d3v_256sq_beams"]
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
            "record_ms": round(r["record_ms"], 5), "record_bytes": r["record_bytes"],
            "roofline": {"bound": "hbm", "kernel": "reverse step (k_adj_* kernels)",
                         "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                         "traffic": None, "bytes_per_launch": r["bytes_per_reverse_step"],
                         "avg_launch_ms": round(r["adjoint_step_ms"], 5)},
            "loss": r["loss"], "dL_dbext": r["dL_dbext"],
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
    wl = picgen.WORKLOADS[args.workload or "3d_64cube_8ppc"]
    precs = ["fp64", "fp32c"] if args.precision == "both" else [args.precision]
    if args.order == 2 or args.interp == "conventional":
        precs = ["fp64"]
    results = {}
    for p in precs:
        results[p] = run_gpu(wl, p, args.steps, args.warmup, args.order, args.interp)
        r = results[p]
        print(f"# {p}: {r['ms_per_step']:.4f} ms/step, particle kernel "
              f"{r['phases']['particles'] / max(1, r['phases']['steps']):.4f} ms, "
              f"gauss_rel {r['diag']['gauss_rel']:.2e}, fallback {r['fallback']:.4f}",
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
                   "ppc": wl.ppc, "dt": wl.dt, "sort_every": wl.sort_every,
                   "precision": main_p, "order": f"{args.order} 1/2", "interp": args.interp,
                   "parallelism": "none (1 GPU)"},
        "roofline": roofline(r, main_p, wl, copy_gbs, args.order, args.interp),
        "phases_ms_per_step": {k: round(v / max(1, r["phases"]["steps"]), 5)
                               for k, v in r["phases"].items() if k != "steps"},
        "checks": {"gauss_rel": r["diag"]["gauss_rel"], "nonfinite": r["diag"]["nonfinite"],
                   "fallback_fraction": r["fallback"]},
    }
    if "fp32c" in results and main_p != "fp32c":
        r32 = results["fp32c"]
        v32 = r32["n"] * 1000.0 / r32["ms_per_step"]
        line["fp32c"] = {"value": round(v32, 1), "ms_per_step": round(r32["ms_per_step"], 5),
                         "speedup_vs_fp64": round(v32 / value, 3),
                         "roofline": roofline(r32, "fp32c", wl, copy_gbs),
                         "gauss_rel": r32["diag"]["gauss_rel"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, order=args.order, interp=args.interp)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
