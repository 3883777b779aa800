"""GPU (HIP, gfx950) vs FP64 CPU oracle for the open x boundary
(pic_grid_desc.xbc = 1): Mur walls at x = 0 and x = nx - 1, the outside cell
layer held at zero, particles absorbed within PIC_ABSORB cells of a wall.
Everything goes through the C ABI.  Tolerances as in test_gpu_parity.py:
FP64 fields and particles to 1e-12 relative; FP32 mode against the FP64
oracle with the loose bounds stated per test.  Absorption is a decision on
the particle's x cell.  In FP64 mode the set of absorbed particles must agree
exactly (positions agree to ~1e-13 cells; the seeded inputs put no particle
that close to a layer edge).  In FP32 mode positions differ from the FP64
oracle by up to ~1e-5 of the box, so a particle that ends a step that close
to a layer edge may be absorbed a step earlier or later: at most 0.2% of the
absorbed set may differ.
"""
import math

import numpy as np
import pytest

import oracle
import picgen

pytestmark = pytest.mark.gpu

ABSORB = 2  # PIC_ABSORB


def _sim(**kw):
    from paper_1101_0809_amd import Sim
    return Sim(**kw)


def _rel(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def _wrapdiff(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


def _beams(nx, ny, nz, dims, ppc, steps, sort_every, drift=0.5, w_th=0.05):
    wl = picgen.Workload("open_beams", nx, ny, nz, dims, 0.45 if dims == 3 else 0.5, ppc,
                         (w_th,) * 3, 0.3, steps, sort_every=sort_every, drift=drift)
    return wl


def _run(wl, precision, source=None, fields=None, ions=True):
    e = picgen.electrons(wl)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision=precision,
               sort_every=wl.sort_every, source=source, fields=fields, xbc="open")
    se = sim.add_species(e.q, e.m, e.n)
    sim.load(se, e.x, e.w, e.weight)
    species = [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m)]
    if ions:
        ion = picgen.ions_like(wl, e)
        si = sim.add_species(ion.q, ion.m, 0, mobile=False)
        sim.load(si, ion.x, ion.w, ion.weight)
        species.append(oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False))
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, source=source, xbc=1), species, fields=fields)
    print(f"open x run: {wl.nx}x{wl.ny}x{wl.nz} dims {wl.dims} {precision} n={e.n} steps={wl.steps}",
          flush=True)
    sim.step(wl.steps)
    st.step(wl.steps)
    return sim, st, e


def _compare(sim, st, wl, field_tol, part_tol, gauss_tol, min_absorbed=1):
    F = sim.fields_numpy()
    for name, sl in (("E", slice(0, 3)), ("B", slice(3, 6))):
        err = _rel(F[sl], st.fields[sl])
        assert err <= field_tol, (name, err)
    nx = wl.nx
    assert np.all(F[1:4, :, :, nx - 1] == 0.0)     # the outside layer holds nothing
    x, w, wt, _ = sim.particles(0)
    sp = st.species[0]
    for a, n in enumerate((wl.nx, wl.ny, wl.nz)[:wl.dims]):
        dx = _wrapdiff(x[a], sp.x[a], n)
        assert np.max(np.abs(dx)) <= part_tol * n, ("x", a, np.max(np.abs(dx)))
    werr = np.max(np.abs(w - sp.w)) / np.max(np.abs(sp.w))
    assert werr <= part_tol, ("w", werr)
    gone_gpu, gone_orc = wt == 0.0, sp.weight == 0.0
    differ = np.count_nonzero(gone_gpu != gone_orc)
    if sim.precision == "fp64":
        assert differ == 0, (np.count_nonzero(gone_gpu), np.count_nonzero(gone_orc))
    else:
        assert differ <= max(2, 2e-3 * np.count_nonzero(gone_orc)), differ
    assert np.count_nonzero(gone_orc) >= min_absorbed
    live = ~gone_orc & ~gone_gpu
    assert np.max(np.abs(wt[live] - sp.weight[live]) / sp.weight[live]) <= (0 if sim.precision == "fp64" else 1e-7)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= gauss_tol, d
    assert d["nonfinite"] == 0
    return d


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_open_x_3d_beams_parity(precision, tols):
    """Two counter-streaming electron beams (w_x = +-0.5, 0.2 cells per step)
    over an immobile background in a 32 x 16 x 16 box with open x walls: over
    24 steps, re-sorted every 6, the beams run into both walls and several
    hundred electrons are absorbed.  Fields, particles, the absorbed set and
    the Gauss drift inside the box against the oracle."""
    wl = _beams(32, 16, 16, 3, 4, 24, 6)
    sim, st, _ = _run(wl, precision)
    _compare(sim, st, wl, *tols, min_absorbed=300)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_open_x_3d_ragged_hot_parity(precision, tols):
    """A hot plasma (w_th = 0.5) on a grid that is not a multiple of the tile
    (21 x 10 x 11), never re-sorted: many electrons leave their tile's region
    and take the migrant path, some of them into the absorbing layers."""
    wl = _beams(21, 10, 11, 3, 3, 12, 0, drift=0.0, w_th=0.5)
    sim, st, _ = _run(wl, precision)
    _compare(sim, st, wl, *tols, min_absorbed=50)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_open_x_2d3v_beams_parity(precision, tols):
    """The 2D3V kernel with open x walls: 48 x 32 cells, beams at w_x = +-0.5,
    30 steps re-sorted every 10."""
    wl = _beams(48, 32, 1, 2, 6, 30, 10)
    sim, st, _ = _run(wl, precision)
    _compare(sim, st, wl, *tols, min_absorbed=300)


@pytest.mark.parametrize("dims", [3, 2])
def test_open_x_laser_in_vacuum_matches_oracle(dims):
    """The plane-wave source in vacuum with open x walls (3D, and 2D3V with
    one z cell): after 160 steps the wave has reached the right wall, which
    absorbs it (Mur), against the oracle's fields and source line."""
    omega = 2 * math.pi / 20
    src = (8, omega, omega, 20.0)
    nz = 8 if dims == 3 else 1
    sim = _sim(nx=64, ny=8, nz=nz, dt=0.45, dims=dims, source=src, xbc="open")
    st = oracle.State(oracle.Grid(64, 8, nz, 0.45, source=src, xbc=1), [])
    sim.step(160)
    st.step(160)
    F = sim.fields_numpy()
    for c in range(6):
        assert np.max(np.abs(F[c] - st.fields[c])) <= 1e-13 * omega, c
    assert np.max(np.abs(sim.aux_line() - st.aux)) <= 1e-13 * omega
    assert np.max(np.abs(F[1][:, :, 40:63])) > 0.9 * omega    # the wave is at the wall


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_open_x_slab_with_laser_parity(precision):
    """The slab workload at reduced size (48 x 16 x 16 cells, cold electrons at
    8 per cell in x in [12, 36), immobile ions) with the laser plane at x = 4
    and open x walls: 60 steps, the laser crosses the slab and leaves."""
    wl = picgen.WORKLOADS["3d_128cube_slab"].scaled(nx=48, ny=16, nz=16, ppc=8, slab=(12, 36),
                                                   steps=60, sort_every=10)
    omega = 2 * math.pi / 20
    tols = (1e-12, 1e-12, 1e-12) if precision == "fp64" else (1e-4, 1e-5, 1e-6)
    sim, st, _ = _run(wl, precision, source=(4, omega, omega, 20.0))
    _compare(sim, st, wl, *tols, min_absorbed=0)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_open_x_diagnostics_match_oracle(precision):
    """pic_diagnostics with open x walls against the oracle's definitions on a
    state where every check is far from zero: random initial E and B, hot
    electrons and a background apart from them, E perturbed after the steps.
    The Gauss drift is the maximum over x cells PIC_ABSORB + 1 .. nx - 3 -
    PIC_ABSORB, div B over x nodes 1 .. nx - 2; the charge counts the
    absorbed electrons no more."""
    import torch
    rng = np.random.Generator(np.random.PCG64(778))
    nx, ny, nz, dt = 19, 10, 9, 0.45
    F0 = np.zeros((9, nz, ny, nx))
    F0[:6] = rng.normal(0.0, 1e-3, (6, nz, ny, nx))
    ne, ni = 3000, 2000
    xe = np.stack([rng.uniform(0, nn, ne) for nn in (nx, ny, nz)])
    we = rng.normal(0.0, 0.4, (3, ne))
    wte = np.full(ne, 0.01)
    xi = np.stack([rng.uniform(0, nn, ni) for nn in (nx, ny, nz)])
    wti = np.full(ni, 0.013)
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=dt, dims=3, precision=precision, sort_every=4, fields=F0, xbc="open")
    se = sim.add_species(-1.0, 1.0, ne)
    sim.load(se, xe, we, wte)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, xi, np.zeros_like(xi), wti)
    x0, _, w0, _ = sim.particles(se)
    sim.step(6)
    F = sim.fields_numpy()
    F[0:3] += rng.normal(0.0, 1e-4, (3, nz, ny, nx))
    sim.fields[0:3].copy_(torch.from_numpy(np.ascontiguousarray(F[0:3])).to(sim.device))
    d = sim.diagnostics()
    x1, _, w1, _ = sim.particles(se)
    assert np.count_nonzero(w1 == 0) > 100
    g = oracle.Grid(nx, ny, nz, dt, xbc=1)
    wti_stored = wti.astype(np.float32).astype(np.float64) if precision == "fp32c" else wti
    ions = oracle.Species(xi, np.zeros_like(xi), wti_stored, q=1.0, m=100.0, mobile=False)
    rho_bg = oracle.State(g, [ions]).rho()
    rho_m0 = oracle.State(g, [oracle.Species(x0, np.zeros_like(x0), w0, q=-1.0)]).rho()
    rho_m1 = oracle.State(g, [oracle.Species(x1, np.zeros_like(x1), w1, q=-1.0)]).rho()
    R0 = oracle.State(g, [], fields=F0).gauss_residual(rho_m0 + rho_bg)
    st1 = oracle.State(g, [], fields=F)
    R1 = st1.gauss_residual(rho_m1 + rho_bg)
    gauss_abs = np.max(np.abs(R1 - R0)[:, :, ABSORB + 1:nx - 2 - ABSORB])
    rho_max = np.max(np.abs(4 * np.pi * rho_m1))
    divb = np.max(np.abs(st1.div_b()[:, :, 1:nx - 1]))
    charge = np.sum(rho_m1 + rho_bg)
    assert gauss_abs > 1e-4 and divb > 1e-4 and abs(charge) > 1.0
    assert np.max(np.abs(R1 - R0)) > gauss_abs     # the excluded cells differ
    assert d["gauss_abs"] == pytest.approx(gauss_abs, rel=1e-12)
    assert d["rho_mobile_max"] == pytest.approx(rho_max, rel=1e-12)
    assert d["divb_max"] == pytest.approx(divb, rel=1e-12)
    assert d["charge"] == pytest.approx(charge, rel=1e-12)
    assert d["nonfinite"] == 0


def test_open_x_rejects_periodic_only_operations():
    """The field-only step, the Poisson start and the adjoint are periodic
    operators: an open-boundary context refuses them with an error."""
    import ctypes

    import torch

    from paper_1101_0809_amd import _lib as L
    sim = _sim(nx=16, ny=8, nz=8, dt=0.45, dims=3, xbc="open")
    e = picgen.electrons(_beams(16, 8, 8, 3, 2, 1, 0))
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    for what in ("b_half", "e_full"):
        with pytest.raises(L.PicError):
            sim.field_solve(what)
    with pytest.raises(L.PicError):
        sim.solve_poisson()
    lam = torch.zeros(9 * sim.ncell, dtype=torch.float64, device=sim.device)
    assert sim.lib.pic_adjoint_seed_field_energy(sim.ctx, ctypes.c_void_p(lam.data_ptr()), None) != 0
    sim.step(2)                                  # stepping itself works
    assert sim.diagnostics()["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_128cube_slab_laser_open_x_fullsize(precision):
    """The full 128^3 slab workload (16,777,216 electrons in x in [32, 96),
    immobile ions, the a0 = 1 laser of 20-cell wavelength from the plane
    x = 8) with open x walls, 300 steps: the laser has crossed the slab and
    reached the right wall.  Checked at full size:
    - the walls follow Mur's update across one more step at every wall point,
      B_wall^{n+1/2} = B_in^{n-1/2} + k (B_in^{n+1/2} - B_wall^{n-1/2});
    - one step of 1500 sampled electrons against the oracle from the GPU's
      own fields;
    - the Gauss drift inside the box, and the empty outside layer.
    The laser's E (about omega = 0.31) is some 300 times the slab's 4 pi rho,
    so in FP64 the drift is set by the rounding of the E updates: each step
    adds a few roundings of |E|-sized values to every E, and div_h E sums six
    of them over dx, so the bar is steps * 16 eps max|E| / dx (absolute)."""
    from test_gpu_parity import _sampled_step_check
    wl = picgen.WORKLOADS["3d_128cube_slab"]
    omega = 2 * math.pi / 20
    src = (8, omega, omega, 20.0)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=128, ny=128, nz=128, dt=wl.dt, dims=3, precision=precision,
               sort_every=wl.sort_every, source=src, xbc="open")
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    del e, ion
    print(f"128^3 slab, open x, {precision}: 299 steps", flush=True)
    sim.step(299)
    B0 = sim.fields_numpy()[3:6].copy()
    g = oracle.Grid(128, 128, 128, wl.dt, xbc=1)
    _sampled_step_check(sim, g, -1.0, 3, (128, 128, 128),
                        1e-12 if precision == "fp64" else 2e-6, nsample=1500)
    F = sim.fields_numpy()
    k = (wl.dt - 1.0) / (wl.dt + 1.0)
    for c in (1, 2):                       # B^y, B^z
        for wall, inside in ((0, 1), (127, 126)):
            want = B0[c][:, :, inside] + k * (F[3 + c][:, :, inside] - B0[c][:, :, wall])
            assert np.max(np.abs(F[3 + c][:, :, wall] - want)) <= 1e-15 * max(1e-30, np.max(np.abs(want))) + 1e-300
    assert np.max(np.abs(F[5][:, :, 120:127])) > 0.3 * omega      # the laser is at the right wall
    assert np.all(F[1:4, :, :, 127] == 0.0)
    d = sim.diagnostics()
    if precision == "fp64":
        assert d["gauss_abs"] <= 300 * 16 * np.finfo(np.float64).eps * np.max(np.abs(F[0:3])), d
    else:
        assert d["gauss_rel"] <= 1e-6, d
    assert d["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_open_x_checkpoint_restore_continue(precision, tmp_path):
    """Save an open-boundary run after 10 steps, restore it into a fresh
    context and continue 10 steps: the same fields, particles and absorbed
    set as 20 steps straight, up to the summation order of the atomics.
    Electrons are absorbed before and after the checkpoint."""
    import torch
    from paper_1101_0809_amd import Sim
    wl = _beams(24, 12, 12, 3, 4, 20, 6)
    e = picgen.electrons(wl)
    sim = _sim(nx=24, ny=12, nz=12, dt=wl.dt, dims=3, precision=precision, sort_every=6, xbc="open")
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    sim.step(10)
    n_half = np.count_nonzero(sim.particles(0)[2] == 0)
    path = tmp_path / "ckpt.pt"
    torch.save(sim.state_dict(), path)
    sim.step(10)
    ref_f = sim.fields_numpy()
    ref_x, ref_w, ref_wt, _ = sim.particles(0)
    sim2 = Sim.from_state_dict(torch.load(path, weights_only=True))
    assert sim2.desc.xbc == 1
    sim2.step(10)
    f = sim2.fields_numpy()
    x, w, wt, _ = sim2.particles(0)
    assert 0 < n_half < np.count_nonzero(ref_wt == 0)
    assert np.array_equal(wt == 0, ref_wt == 0)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for c in range(6):
        assert _rel(f[c], ref_f[c]) < tol
    assert np.max(np.abs(w - ref_w)) < tol * np.max(np.abs(ref_w))
    assert np.max(np.abs(_wrapdiff(x, ref_x, np.array([[24], [12], [12]])))) < tol * 24
