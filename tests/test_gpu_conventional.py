"""GPU path with the conventional uniform-order interpolation of Eq. wrong1
(the comparison of Section 5) against the FP64 oracle with the same
interpolation, through the C ABI.  Same tolerances as the alternating-order
parity tests: 1e-12 relative on fields and particle states, Gauss drift at
most 1e-12 of max |4 pi rho_e|."""
import numpy as np
import pytest

import oracle
import picgen

pytestmark = pytest.mark.gpu


def _sim(interp="conventional", **kw):
    from paper_1101_0809_amd import Sim
    return Sim(interp=interp, **kw)


def _rel(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def _wrapdiff(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


def _run_pair(wl, steps):
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, sort_every=wl.sort_every, bext=wl.bext)
    sim.add_species(e.q, e.m, e.n)
    sim.load(0, e.x, e.w, e.weight)
    sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(1, ion.x, ion.w, ion.weight)
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext, interp=1),
                      [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m),
                       oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False)])
    sim.step(steps)
    st.step(steps)
    return sim, st


def _compare(sim, st, wl, tol=1e-12):
    F = sim.fields_numpy()
    for sl in (slice(0, 3), slice(3, 6)):
        assert _rel(F[sl], st.fields[sl]) <= tol
    x, w, _, _ = sim.particles(0)
    sp = st.species[0]
    for a, n in enumerate((wl.nx, wl.ny, wl.nz)[:wl.dims]):
        assert np.max(np.abs(_wrapdiff(x[a], sp.x[a], n))) <= tol * n
    assert np.max(np.abs(w - sp.w)) / np.max(np.abs(sp.w)) <= tol
    d = sim.diagnostics()
    assert d["gauss_rel"] <= 1e-12, d
    assert d["nonfinite"] == 0


def test_conventional_2d3v_32x32_parity():
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(sort_every=10)
    sim, st = _run_pair(wl, wl.steps)
    _compare(sim, st, wl)


def test_conventional_3d_small_parity():
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=16, ny=16, nz=16, steps=20, sort_every=5)
    sim, st = _run_pair(wl, wl.steps)
    _compare(sim, st, wl)


def test_conventional_3d_ragged_hot_parity():
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=13, ny=10, nz=11, w_th=(0.5, 0.5, 0.5), ppc=3,
                                                  steps=12, sort_every=0)
    sim, st = _run_pair(wl, wl.steps)
    assert sim.fallback_fraction() > 0.0
    _compare(sim, st, wl)


def test_conventional_small_grids():
    for wl in (picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(nx=7, ny=5, steps=15, sort_every=4),
               picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=5, ny=4, nz=6, ppc=4, steps=10, sort_every=3)):
        sim, st = _run_pair(wl, wl.steps)
        _compare(sim, st, wl)


def test_conventional_64cube_fullsize_sampled():
    """Full 64^3 x 8 per cell after 20 steps: one more step checked on a
    sample of particles against the oracle's conventional gather and push on
    the GPU's own pre-step fields."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"]
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=64, ny=64, nz=64, dt=wl.dt, dims=3, sort_every=10)
    sim.add_species(e.q, e.m, e.n)
    sim.load(0, e.x, e.w, e.weight)
    sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(1, ion.x, ion.w, ion.weight)
    sim.step(20)
    fields = sim.fields_numpy()
    x0, w0, _, ids = sim.particles(0)
    sim.step(1)
    x1, w1, _, ids1 = sim.particles(0)
    assert np.array_equal(ids, ids1)
    g = oracle.Grid(64, 64, 64, wl.dt, interp=1)
    bn = fields.copy()
    oracle.half_b(g, bn)
    rng = np.random.Generator(np.random.PCG64(97))
    for p in rng.choice(e.n, 3000, replace=False):
        E, B = oracle.gather(g, bn, x0[:, p])
        wn = oracle.push(-1.0, wl.dt, 1.0, E, B, w0[:, p])
        xn = x0[:, p] + oracle.displacement(g, wn)
        assert np.max(np.abs(wn - w1[:, p])) <= 1e-12 * max(1e-3, np.max(np.abs(wn)))
        assert np.max(np.abs(_wrapdiff(xn, x1[:, p], 64))) <= 1e-12 * 64
    d = sim.diagnostics()
    assert d["gauss_rel"] <= 1e-12, d
    sim.close()


def test_energy_defect_conventional_versus_alternating_on_gpu():
    """Section 5, Fig. 2 (left) at reduced size on the GPU: thermal plasma
    with v_Te = 0.05 c, 2 electrons per cell, mesh = Debye length, c dt = dx/2,
    co-located ions, 32^3 cells, 200 steps.  The conventional interpolation's
    total-energy defect is far above the alternating order's (the paper: two
    orders of magnitude); the energy counted is kinetic plus field energy."""
    wl = picgen.Workload("x1", 32, 32, 32, 3, 0.5, 2, (0.05,) * 3, 0.05, 200, sort_every=10, seed=11)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    out = {}
    for interp in ("alternating", "conventional"):
        sim = _sim(interp=interp, nx=32, ny=32, nz=32, dt=wl.dt, dims=3, sort_every=10)
        sim.add_species(e.q, e.m, e.n)
        sim.load(0, e.x, e.w, e.weight)
        sim.add_species(ion.q, ion.m, 0, mobile=False)
        sim.load(1, ion.x, ion.w, ion.weight)
        d0 = sim.diagnostics()
        tot0 = d0["kinetic"] + d0["field_e"] + d0["field_b"]
        sim.step(wl.steps)
        d = sim.diagnostics()
        out[interp] = abs(d["kinetic"] + d["field_e"] + d["field_b"] - tot0) / tot0
        assert d["gauss_rel"] <= 1e-12
        sim.close()
    assert out["conventional"] > 30 * out["alternating"], out
