"""GPU adjoint (pic_adjoint_seed_field_energy, pic_adjoint_step) against the
reference gradient of oracle/adjoint.py (torch autograd through a CPU FP64
restatement of the step, itself pinned to the C oracle and to its central
differences).

Tolerance.  The GPU forward agrees with the oracle to ~1e-15 relative per
step; the adjoint evaluates the same derivatives in another order (forward-
mode dual numbers or separable partial sums per particle against reverse-mode
autograd), so each
gradient component is compared with a bar of 1e-9 of the largest component
of its array, far above rounding and far below any dropped or mis-signed
term (those move components by O(1) of the scale).
"""
import numpy as np
import pytest
import torch

import oracle.adjoint as ad
import picgen

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _gpu_grad(box, dims, dt, x, w, weight, bext, steps, every, sort_every=3, ions=False):
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd.adjoint import field_energy_grad
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=dims, sort_every=sort_every, bext=bext)
    sim.add_species(-1.0, 1.0, capacity=weight.size)
    sim.load(0, x, w, weight)
    if ions:
        sim.add_species(1.0, 1836.0, capacity=weight.size, mobile=False)
        sim.load(1, x, np.zeros_like(w), weight)
    L, gx, gw, gb = field_energy_grad(sim, steps, every=every)
    torch.cuda.synchronize()
    out = (L, gx[0].cpu().numpy(), gw[0].cpu().numpy(), gb.cpu().numpy())
    sim.close()
    return out


def _close(a, b, tol=TOL):
    scale = np.max(np.abs(b))
    err = np.max(np.abs(a - b))
    assert err <= tol * scale, (err, scale)


def _fields(shape, seed, amp):
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((9,) + shape)
    f[:6] = rng.normal(0.0, amp, (6,) + shape)
    return f


def test_seed_matches_reference():
    """pic_adjoint_seed_field_energy on random fields (ragged 11 x 7 x 5)."""
    from paper_1101_0809_amd import Sim
    nx, ny, nz = 11, 7, 5
    f = _fields((nz, ny, nx), 71, 0.3)
    sim = Sim(nx=nx, ny=ny, nz=nz, dt=0.45, dims=3, fields=f)
    lam = torch.empty(6 * sim.ncell, dtype=torch.float64, device="cuda:0")
    sim.adjoint_seed_field_energy(lam)
    got = lam.cpu().numpy().reshape(6, nz, ny, nx)
    gE, gB = ad.field_energy_grad_fields(ad.Grid(nx, ny, nz, 0.45), f[:3], f[3:6])
    _close(got[:3], gE, 1e-13)
    _close(got[3:], gB, 1e-13)
    sim.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_step_vjp_matches_reference(dims):
    """One pic_adjoint_step with random adjoints, random fields and particles
    spanning several tiles (ragged counts and grid) against the oracle's
    one-step vector-Jacobian product; ids are permuted by a sort first."""
    from paper_1101_0809_amd import Sim
    box = (21, 18, 1) if dims == 2 else (10, 9, 11)
    dt = 0.5 if dims == 2 else 0.45
    n = 1501 if dims == 2 else 1303
    x, w, weight = picgen.beams(box, n, 80 + dims, w_th=0.3, drift=0.2, dims=dims)
    shape = (box[2], box[1], box[0])
    f = _fields(shape, 90 + dims, 0.05)
    bext = (0.03, -0.02, 0.05)
    rng = np.random.Generator(np.random.PCG64(100 + dims))
    lam = [rng.normal(size=(3,) + shape), rng.normal(size=(3,) + shape),
           rng.normal(size=(3, n)), rng.normal(size=(3, n))]
    if dims == 2:
        lam[2][2] = 0.0
    ref = ad.step_vjp(ad.Grid(*box, dt), f[:3], f[3:6], x, w, weight, -1.0, 1.0, bext, *lam)
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=dims, bext=bext, fields=f)
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    sim.sort()
    dev = torch.device("cuda:0")
    lf = torch.tensor(np.concatenate([lam[0], lam[1]]).reshape(-1), device=dev)
    lx = torch.tensor(lam[2], device=dev)
    lw = torch.tensor(lam[3], device=dev)
    lb = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step(lf, [lx], [lw], lb)
    got = lf.cpu().numpy().reshape((6,) + shape)
    _close(got[:3], ref[0], 1e-12)
    _close(got[3:], ref[1], 1e-12)
    _close(lx.cpu().numpy()[:dims], ref[2][:dims], 1e-12)
    _close(lw.cpu().numpy(), ref[3], 1e-12)
    _close(lb.cpu().numpy(), ref[4], 1e-12)
    sim.close()


def test_step_vjp_crowded_tile_scatters_in_storage_order():
    """3D reverse step where one 8^3 tile holds 60000 particles (64 x 64 x 8
    cells, 8 blocks per tile: 7500 per block, more than a block's class
    queue), beside 3000 particles spread over the other tiles, which use the
    queue.  The crowded tile's blocks scatter lambda_Ep, lambda_Bp in storage
    order.  Against the oracle's one-step vector-Jacobian product; the bar is
    1e-11 of each array's largest component (about 3000 particle terms sum
    into one accumulator cell)."""
    from paper_1101_0809_amd import Sim
    box, dt = (64, 64, 8), 0.45
    rng = np.random.Generator(np.random.PCG64(515))
    nc, ns = 60000, 3000
    x = np.concatenate([rng.uniform(0.0, 8.0, (3, nc)),
                        np.stack([rng.uniform(0, box[a], ns) for a in range(3)])], axis=1)
    n = nc + ns
    w = rng.normal(0.0, 0.1, (3, n))
    weight = np.full(n, 1e-4)
    shape = (box[2], box[1], box[0])
    f = _fields(shape, 516, 0.05)
    bext = (0.03, -0.02, 0.05)
    lam = [rng.normal(size=(3,) + shape), rng.normal(size=(3,) + shape),
           rng.normal(size=(3, n)), rng.normal(size=(3, n))]
    ref = ad.step_vjp(ad.Grid(*box, dt), f[:3], f[3:6], x, w, weight, -1.0, 1.0, bext, *lam)
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=3, bext=bext, fields=f)
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    sim.sort()
    dev = torch.device("cuda:0")
    lf = torch.tensor(np.concatenate([lam[0], lam[1]]).reshape(-1), device=dev)
    lx = torch.tensor(lam[2], device=dev)
    lw = torch.tensor(lam[3], device=dev)
    lb = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step(lf, [lx], [lw], lb)
    got = lf.cpu().numpy().reshape((6,) + shape)
    _close(got[:3], ref[0], 1e-11)
    _close(got[3:], ref[1], 1e-11)
    _close(lx.cpu().numpy(), ref[2], 1e-11)
    _close(lw.cpu().numpy(), ref[3], 1e-11)
    _close(lb.cpu().numpy(), ref[4], 1e-11)
    sim.close()


def test_step_vjp_particles_off_their_tile():
    """3D reverse step of a state six steps after its sort (hot beams, 24 x 16
    x 16 cells, 12 tiles, no re-sort): a few percent of the particles lie more
    than one cell outside the tile of their sorted slot, where the tile
    kernel queues them and runs them on global memory after the others.
    Against the oracle's one-step vector-Jacobian product of that state."""
    from paper_1101_0809_amd import Sim
    box, dt, n = (24, 16, 16), 0.45, 4000
    x, w, weight = picgen.beams(box, n, 91, w_th=0.5, drift=0.3, dims=3)
    shape = (box[2], box[1], box[0])
    f = _fields(shape, 92, 0.05)
    bext = (0.02, 0.01, -0.03)
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=3, bext=bext, fields=f)
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    sim.sort()
    sim.step(6)
    F = sim.fields_numpy()
    xs, ws, wts, ids = sim.particles(0)
    assert np.array_equal(ids, np.arange(n))
    # the state really has particles more than one cell off the tile they
    # were sorted into (the sort put each in the tile of its load position),
    # with the kernel's periodic offset convention
    rel = np.floor(xs) - np.floor(x / 8) * 8
    for ax, nax in enumerate(box):
        rel[ax] = np.where(rel[ax] > nax // 2, rel[ax] - nax, rel[ax])
        rel[ax] = np.where(rel[ax] < -(nax // 2), rel[ax] + nax, rel[ax])
    off = int(((rel < -1) | (rel > 8)).any(axis=0).sum())
    assert off >= 20, off
    rng = np.random.Generator(np.random.PCG64(93))
    lam = [rng.normal(size=(3,) + shape), rng.normal(size=(3,) + shape),
           rng.normal(size=(3, n)), rng.normal(size=(3, n))]
    ref = ad.step_vjp(ad.Grid(*box, dt), F[:3], F[3:6], xs, ws, wts, -1.0, 1.0, bext, *lam)
    dev = torch.device("cuda:0")
    lf = torch.tensor(np.concatenate([lam[0], lam[1]]).reshape(-1), device=dev)
    lx = torch.tensor(lam[2], device=dev)
    lw = torch.tensor(lam[3], device=dev)
    lb = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step(lf, [lx], [lw], lb)
    got = lf.cpu().numpy().reshape((6,) + shape)
    _close(got[:3], ref[0], 1e-12)
    _close(got[3:], ref[1], 1e-12)
    _close(lx.cpu().numpy(), ref[2], 1e-12)
    _close(lw.cpu().numpy(), ref[3], 1e-12)
    _close(lb.cpu().numpy(), ref[4], 1e-12)
    sim.close()


def test_step_vjp_off_tile_queue_overflow():
    """3D reverse step of a tile whose off-tile queue overflows: 12,000
    electrons loaded into one 8^3 tile of a 64^3 grid (512 tiles, so one
    workgroup per tile) near its +x face, beamed along +x at w_x = 3 (0.43
    cells per step), sorted, then stepped 6 times without a re-sort.  About
    four in five end more than one cell outside the tile, more than the
    7168 entries of the workgroup's queue, so the rest run their global form
    inline in phase 1.  Against the oracle's one-step vector-Jacobian
    product of that state."""
    from paper_1101_0809_amd import Sim
    box, dt, n = (64, 64, 64), 0.45, 12000
    rng = np.random.Generator(np.random.PCG64(97))
    x = np.stack([6.0 + 2.0 * rng.random(n), 8.0 * rng.random(n), 8.0 * rng.random(n)])
    w = rng.normal(0.0, 0.05, (3, n))
    w[0] += 3.0
    weight = np.full(n, 1e-6)  # a light beam: its own field barely deflects it
    shape = (box[2], box[1], box[0])
    f = _fields(shape, 98, 0.05)
    bext = (0.01, -0.02, 0.03)
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=3, bext=bext, fields=f, sort_every=0)
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    sim.sort()
    sim.step(6)
    F = sim.fields_numpy()
    xs, ws, wts, ids = sim.particles(0)
    assert np.array_equal(ids, np.arange(n))
    # every particle was sorted into tile 0; count those beyond its region
    # (cells -1 .. 8 on each axis)
    off = int(((np.floor(xs) < -1) | (np.floor(xs) > 8)).any(axis=0).sum())
    assert off > 7168 + 1000, off
    lam = [rng.normal(size=(3,) + shape), rng.normal(size=(3,) + shape),
           rng.normal(size=(3, n)), rng.normal(size=(3, n))]
    ref = ad.step_vjp(ad.Grid(*box, dt), F[:3], F[3:6], xs, ws, wts, -1.0, 1.0, bext, *lam)
    dev = torch.device("cuda:0")
    lf = torch.tensor(np.concatenate([lam[0], lam[1]]).reshape(-1), device=dev)
    lx = torch.tensor(lam[2], device=dev)
    lw = torch.tensor(lam[3], device=dev)
    lb = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step(lf, [lx], [lw], lb)
    got = lf.cpu().numpy().reshape((6,) + shape)
    _close(got[:3], ref[0], 1e-12)
    _close(got[3:], ref[1], 1e-12)
    _close(lx.cpu().numpy(), ref[2], 1e-12)
    _close(lw.cpu().numpy(), ref[3], 1e-12)
    _close(lb.cpu().numpy(), ref[4], 1e-12)
    sim.close()


CASES = {
    # 2D3V beams in B_z, several sorts and checkpoint segments
    "2d_8x8": dict(box=(8, 8, 1), dims=2, dt=0.5, n=64, seed=17, w_th=0.05, drift=0.2,
                   bext=(0.0, 0.0, 0.05), steps=10, every=4),
    # 3D with every component of B_ext non-zero
    "3d_6x5x4": dict(box=(6, 5, 4), dims=3, dt=0.45, n=48, seed=8, w_th=0.2, drift=0.0,
                     bext=(0.02, -0.03, 0.05), steps=8, every=3),
    # several 8x8 tiles and a ragged tail of particles
    "2d_32x24": dict(box=(32, 24, 1), dims=2, dt=0.5, n=3001, seed=21, w_th=0.1, drift=0.15,
                     bext=(0.01, 0.0, 0.08), steps=12, every=5),
    "3d_12x10x9": dict(box=(12, 10, 9), dims=3, dt=0.45, n=2161, seed=22, w_th=0.1, drift=0.1,
                       bext=(0.0, 0.04, 0.02), steps=6, every=4),
}


@pytest.mark.parametrize("mode", ["checkpoints", "tape"])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_reference_gradient(name, mode):
    """Checkpoints: state copies every few steps, segments re-run in the
    reverse pass; tape: a record of every step taken in the forward pass."""
    c = CASES[name]
    x, w, weight = picgen.beams(c["box"], c["n"], c["seed"], w_th=c["w_th"], drift=c["drift"],
                                dims=c["dims"])
    g = ad.Grid(*c["box"], c["dt"])
    L_ref, gw_ref, gb_ref, gx_ref = ad.loss_and_grad(g, x, w, weight, -1.0, 1.0, c["bext"], c["steps"])
    L, gx, gw, gb = _gpu_grad(c["box"], c["dims"], c["dt"], x, w, weight, c["bext"], c["steps"],
                              c["every"] if mode == "checkpoints" else None)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    _close(gw, gw_ref)
    _close(gx[: c["dims"]], gx_ref[: c["dims"]])
    if c["dims"] == 2:
        assert np.max(np.abs(gx[2])) == 0.0
    _close(gb, gb_ref)


def test_adjoint_with_immobile_ions_and_checkpoint_spacing():
    """An immobile neutralising species adds charge but no adjoint; the
    gradient does not depend on the checkpoint spacing (one copy per step vs
    one for the whole run)."""
    c = CASES["2d_8x8"]
    x, w, weight = picgen.beams(c["box"], c["n"], c["seed"], w_th=c["w_th"], drift=c["drift"], dims=2)
    g = ad.Grid(*c["box"], c["dt"])
    ref = ad.loss_and_grad(g, x, w, weight, -1.0, 1.0, c["bext"], c["steps"])
    a = _gpu_grad(c["box"], 2, c["dt"], x, w, weight, c["bext"], c["steps"], every=1, ions=True)
    b = _gpu_grad(c["box"], 2, c["dt"], x, w, weight, c["bext"], c["steps"], every=100, ions=True,
                  sort_every=0)
    for got in (a, b):
        assert abs(got[0] - ref[0]) <= 1e-12 * ref[0]
        _close(got[2], ref[1])
        _close(got[3], ref[2])
        _close(got[1][:2], ref[3][:2])


def test_autograd_function_and_central_difference_of_gpu_forward():
    """torch.autograd through paper_1101_0809_amd.adjoint.field_energy gives
    the driver's gradient; dL/dB_ext,z matches central differences of the
    GPU forward itself."""
    from paper_1101_0809_amd.adjoint import field_energy
    c = CASES["2d_8x8"]
    x, w, weight = picgen.beams(c["box"], c["n"], c["seed"], w_th=c["w_th"], drift=c["drift"], dims=2)
    grid = dict(nx=8, ny=8, nz=1, dt=c["dt"], dims=2, sort_every=3)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev, requires_grad=True)
    wt = torch.tensor(w, device=dev, requires_grad=True)
    bt = torch.tensor(c["bext"], dtype=torch.float64, requires_grad=True)
    L = field_energy(xt, wt, torch.tensor(weight, device=dev), bt, grid, c["steps"], every=4)
    gx, gw, gb = torch.autograd.grad(3.0 * L, (xt, wt, bt))
    L0, gx0, gw0, gb0 = _gpu_grad(c["box"], 2, c["dt"], x, w, weight, c["bext"], c["steps"], 4)
    assert abs(float(L.detach()) - L0) <= 1e-13 * L0
    _close(gw.cpu().numpy(), 3.0 * gw0)
    _close(gx.cpu().numpy()[:2], 3.0 * gx0[:2])
    _close(gb.numpy(), 3.0 * gb0)
    h = 1e-6
    Lp = float(field_energy(xt.detach(), wt.detach(), torch.tensor(weight, device=dev),
                            bt.detach() + torch.tensor([0.0, 0.0, h], dtype=torch.float64),
                            grid, c["steps"]))
    Lm = float(field_energy(xt.detach(), wt.detach(), torch.tensor(weight, device=dev),
                            bt.detach() - torch.tensor([0.0, 0.0, h], dtype=torch.float64),
                            grid, c["steps"]))
    fd = (Lp - Lm) / (2 * h)
    assert abs(gb0[2] - fd) <= 1e-6 * abs(fd), (gb0[2], fd)


@pytest.mark.parametrize("dims", [2, 3])
def test_record_step_equals_context_step(dims):
    """pic_adjoint_step_record on a record of the context's state gives what
    pic_adjoint_step gives on the context itself, for a sorted state and for
    the unsorted state right after loading."""
    from paper_1101_0809_amd import Sim
    box = (21, 18, 1) if dims == 2 else (10, 9, 11)
    n = 1501 if dims == 2 else 1303
    x, w, weight = picgen.beams(box, n, 110 + dims, w_th=0.3, drift=0.2, dims=dims)
    shape = (box[2], box[1], box[0])
    sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=0.45, dims=dims, bext=(0.01, 0.02, 0.03),
              fields=_fields(shape, 120 + dims, 0.05), sort_every=4)
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64(130 + dims))
    lam0 = [torch.tensor(rng.normal(size=6 * sim.ncell), device=dev),
            torch.tensor(rng.normal(size=(3, n)), device=dev),
            torch.tensor(rng.normal(size=(3, n)), device=dev)]
    for stepped in (0, 2):
        sim.step(stepped)
        outs = []
        for use_record in (False, True):
            lf, lx, lw = (t.clone() for t in lam0)
            lb = torch.zeros(3, dtype=torch.float64, device=dev)
            if use_record:
                rec = torch.empty(sim.adjoint_record_bytes(), dtype=torch.uint8, device=dev)
                sim.adjoint_record(rec)
                sim.step(1)  # the context moves on; the record keeps the state
                sim.adjoint_step_record(rec, lf, [lx], [lw], lb)
            else:
                sim.adjoint_step(lf, [lx], [lw], lb)
            outs.append([t.cpu().numpy() for t in (lf, lx, lw, lb)])
        for a, b in zip(*outs):
            _close(a, b, 1e-13)
    rec = torch.empty(sim.adjoint_record_bytes() - 256, dtype=torch.uint8, device=dev)
    from paper_1101_0809_amd._lib import PicError
    with pytest.raises(PicError):
        sim.adjoint_record(rec)
    sim.close()


def test_ordered_step_and_reorder():
    """pic_adjoint_reorder from id order to a record's storage order is the
    gather by the record's ids and back again the identity; the ordered
    reverse step on reordered adjoints equals the id-order step."""
    from paper_1101_0809_amd import Sim
    box, n = (21, 18, 1), 1501
    x, w, weight = picgen.beams(box, n, 140, w_th=0.3, drift=0.2, dims=2)
    sim = Sim(nx=21, ny=18, nz=1, dt=0.5, dims=2, sort_every=3, fields=_fields((1, 18, 21), 141, 0.05))
    sim.add_species(-1.0, 1.0, capacity=n)
    sim.load(0, x, w, weight)
    sim.step(2)
    dev = torch.device("cuda:0")
    rec = torch.empty(sim.adjoint_record_bytes(), dtype=torch.uint8, device=dev)
    sim.adjoint_record(rec)
    _, _, _, ids = sim.particles(0, raw=True)
    rng = np.random.Generator(np.random.PCG64(142))
    lx0 = torch.tensor(rng.normal(size=(3, n)), device=dev)
    lw0 = torch.tensor(rng.normal(size=(3, n)), device=dev)
    lf0 = torch.tensor(rng.normal(size=6 * sim.ncell), device=dev)
    ox, ow = torch.empty_like(lx0), torch.empty_like(lw0)
    sim.adjoint_reorder(None, rec, [lx0], [lw0], [ox], [ow])
    assert np.array_equal(ox.cpu().numpy(), lx0.cpu().numpy()[:, ids])
    assert np.array_equal(ow.cpu().numpy(), lw0.cpu().numpy()[:, ids])
    bx, bw = torch.empty_like(lx0), torch.empty_like(lw0)
    sim.adjoint_reorder(rec, None, [ox], [ow], [bx], [bw])
    assert torch.equal(bx, lx0) and torch.equal(bw, lw0)
    # id-order step vs ordered step on the reordered adjoints
    lf_a, lx_a, lw_a = lf0.clone(), lx0.clone(), lw0.clone()
    lb_a = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step_record(rec, lf_a, [lx_a], [lw_a], lb_a)
    lf_b = lf0.clone()
    lb_b = torch.zeros(3, dtype=torch.float64, device=dev)
    sim.adjoint_step_record(rec, lf_b, [ox], [ow], lb_b, ordered=True)
    sim.adjoint_reorder(rec, None, [ox], [ow], [bx], [bw])
    for a, b in ((lf_a, lf_b), (lx_a, bx), (lw_a, bw), (lb_a, lb_b)):
        _close(a.cpu().numpy(), b.cpu().numpy(), 1e-13)
    from paper_1101_0809_amd._lib import PicError
    with pytest.raises(PicError):
        sim.adjoint_reorder(None, rec, [ox], [ow], [ox], [bw])  # in place
    sim.close()


def test_adjoint_rejects_fp32_mode():
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd._lib import PicError
    sim = Sim(nx=8, ny=8, nz=1, dt=0.5, dims=2, precision="fp32c")
    lam = torch.zeros(6 * 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(PicError):
        sim.adjoint_seed_field_energy(lam)
    sim.close()


def test_full_size_2d_beams_gradient_matches_central_differences():
    """The differentiable workload at its full size (2D3V 256 x 256, 1,048,576
    electrons in two beams drifting at +-0.2 c, B_z = 0.02, 200 steps): the
    tape gradient against central differences (h = 1e-6) of the GPU forward
    pass on B_z, on 32 random momentum components and along 8 random
    directions of all momenta, and against the checkpointed gradient (every
    20 steps).  Reruns of the forward pass agree to the last bit or two (the
    order of LDS atomics may change), far below what h = 1e-6 resolves, so
    the differences carry truncation error: measured about 1e-5 relative on
    B_z and the directions and 2e-7 of the largest component on single
    components."""
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd.adjoint import field_energy_grad
    wl = picgen.WORKLOADS["2d3v_256sq_beams"]
    e = picgen.electrons(wl)

    def make(w=None, bext=None):
        sim = Sim(nx=wl.nx, ny=wl.ny, nz=1, dt=wl.dt, dims=2, sort_every=wl.sort_every,
                  bext=wl.bext if bext is None else tuple(bext))
        sim.add_species(-1.0, 1.0, e.n)
        sim.load(0, e.x, e.w if w is None else w, e.weight)
        return sim

    def loss(w=None, bext=None):
        sim = make(w, bext)
        sim.step(wl.steps)
        d = sim.diagnostics()
        sim.close()
        return d["field_e"] + d["field_b"]

    sim = make()
    L, gx, gw, gb = field_energy_grad(sim, wl.steps)
    sim.close()
    gw = gw[0].cpu().numpy()
    gb = gb.cpu().numpy()
    sim = make()
    L2, _, gw2, gb2 = field_energy_grad(sim, wl.steps, every=20)
    sim.close()
    assert abs(L2 - L) <= 1e-12 * L
    _close(gw2[0].cpu().numpy(), gw, 1e-10)
    _close(gb2.cpu().numpy(), gb, 1e-10)
    assert abs(loss() - L) <= 1e-12 * L
    h = 1e-6
    b = np.array(wl.bext)
    fd = (loss(bext=b + [0, 0, h]) - loss(bext=b - [0, 0, h])) / (2 * h)
    assert abs(gb[2] - fd) <= 1e-4 * abs(fd), (gb[2], fd)
    scale = np.max(np.abs(gw))
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(32):
        c, p = int(rng.integers(0, 3)), int(rng.integers(0, e.n))
        wp, wm = e.w.copy(), e.w.copy()
        wp[c, p] += h
        wm[c, p] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert abs(gw[c, p] - fd) <= 1e-5 * scale, (c, p, gw[c, p], fd)
    for _ in range(8):
        d = rng.normal(size=e.w.shape)
        d /= np.linalg.norm(d)
        fd = (loss(e.w + h * d) - loss(e.w - h * d)) / (2 * h)
        an = float(np.sum(gw * d))
        assert abs(an - fd) <= 1e-4 * abs(an), (an, fd)


@pytest.mark.parametrize("dims", [2, 3])
def test_adjoint_two_mobile_species(dims):
    """Electrons and mobile ions (q = +1, m = 25): per-species particle
    adjoints and dL/dB_ext against the reference gradient, tape and
    checkpoint modes."""
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd.adjoint import field_energy_grad
    box = (16, 12, 1) if dims == 2 else (8, 7, 6)
    dt = 0.5 if dims == 2 else 0.45
    xe, we, wte = picgen.beams(box, 300, 51, w_th=0.1, drift=0.15, dims=dims)
    xi, wi, wti = picgen.beams(box, 200, 52, w_th=0.02, dims=dims)
    bext = (0.01, 0.0, 0.04)
    L_ref, grads, gb_ref = ad.loss_and_grad_species(
        ad.Grid(*box, dt), [(xe, we, wte, -1.0, 1.0), (xi, wi, wti, 1.0, 25.0)], bext, 10)
    for every in (None, 3):
        sim = Sim(nx=box[0], ny=box[1], nz=box[2], dt=dt, dims=dims, sort_every=4, bext=bext)
        sim.add_species(-1.0, 1.0, capacity=300)
        sim.load(0, xe, we, wte)
        sim.add_species(1.0, 25.0, capacity=200)
        sim.load(1, xi, wi, wti)
        L, gx, gw, gb = field_energy_grad(sim, 10, every=every)
        assert abs(L - L_ref) <= 1e-12 * L_ref
        for k in range(2):
            _close(gw[k].cpu().numpy(), grads[k][0])
            _close(gx[k].cpu().numpy()[:dims], grads[k][1][:dims])
        _close(gb.cpu().numpy(), gb_ref)
        sim.close()
