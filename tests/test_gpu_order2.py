"""GPU path at alternating order 2 1/2 (Section 4.5) against the FP64 oracle
at the same order, through the C ABI.

The tolerances are those of the order-1 1/2 parity tests (test_gpu_parity):
the GPU evaluates the same formulas in another order and with fused
multiply-adds, so single operations differ in the last bit; fields and
particle states agree to 1e-12 relative over the runs below, and the Gauss
drift stays below 1e-12 of max |4 pi rho_e|.
"""
import numpy as np
import pytest

import oracle
import picgen

pytestmark = pytest.mark.gpu


def _sim(**kw):
    from paper_1101_0809_amd import Sim
    return Sim(order=2, **kw)


def _rel(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def _wrapdiff(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


@pytest.mark.parametrize("dims", [3, 2])
def test_deposit_order2_matches_oracle(dims):
    """pic_deposit_J at order 2 1/2 for many random moves (several tiles,
    moves across the periodic boundary, a ragged count) equals the oracle's
    current at the same order."""
    n = 16
    nz = n if dims == 3 else 1
    sim = _sim(nx=n, ny=12, nz=nz, dt=0.41, dims=dims, dx=1.1, dy=0.9, dz=1.0)
    g = oracle.Grid(n, 12, nz, 0.41, dx=1.1, dy=0.9, dz=1.0, order=2)
    x0, x1 = picgen.random_moves(1237, seed=25, box=(n, 12, nz), max_step=0.9)
    if dims == 2:
        x1[2] = x0[2] + (x1[2] - x0[2]) * 0.5
    q = np.linspace(0.5, 1.5, x0.shape[1])
    J = sim.deposit(x0, x1, q).cpu().numpy()
    ref = np.zeros_like(J)
    for p in range(x0.shape[1]):
        oracle.deposit(g, x0[:, p], x1[:, p], q[p], J=ref)
    assert _rel(J, ref) <= 1e-13
    sim.close()


def _run_pair(wl, steps, ions=True):
    e = picgen.electrons(wl)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, sort_every=wl.sort_every, bext=wl.bext)
    sim.add_species(e.q, e.m, e.n)
    sim.load(0, e.x, e.w, e.weight)
    species = [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m)]
    if ions:
        ion = picgen.ions_like(wl, e)
        sim.add_species(ion.q, ion.m, 0, mobile=False)
        sim.load(1, ion.x, ion.w, ion.weight)
        species.append(oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False))
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext, order=2), species)
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


def test_order2_2d3v_32x32_parity():
    """2D3V 32x32, 4 electrons per cell, 100 steps, re-sorted every 10."""
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(sort_every=10)
    sim, st = _run_pair(wl, wl.steps)
    _compare(sim, st, wl)


def test_order2_3d_small_parity():
    """3D 16^3 (8 tiles) x 8 per cell, 20 steps, re-sorted every 5."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=16, ny=16, nz=16, steps=20, sort_every=5)
    sim, st = _run_pair(wl, wl.steps)
    _compare(sim, st, wl)


def test_order2_3d_ragged_hot_parity():
    """Partial tiles, hot plasma without re-sort: many particles leave their
    tile and take the global-memory path."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=13, ny=10, nz=11, w_th=(0.5, 0.5, 0.5), ppc=3,
                                                  steps=12, sort_every=0)
    sim, st = _run_pair(wl, wl.steps)
    assert sim.fallback_fraction() > 0.0
    _compare(sim, st, wl)


def test_order2_small_grid_wraps_onto_itself():
    """A 2D grid smaller than the kernel's LDS regions (they cover cells more
    than once) and a 3D grid of 5 x 4 x 6 cells."""
    for wl in (picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(nx=7, ny=5, steps=15, sort_every=4),
               picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=5, ny=4, nz=6, ppc=4, steps=10, sort_every=3)):
        sim, st = _run_pair(wl, wl.steps)
        _compare(sim, st, wl)


def test_order2_64cube_fullsize_sampled():
    """Full 64^3 x 8 per cell (2,097,152 electrons) at order 2 1/2: after 20
    steps (two re-sorts) one more step is checked particle by particle on a
    sample against the oracle's gather and push at the same order, using the
    GPU's own pre-step fields; the Gauss drift holds over the whole grid."""
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
    g = oracle.Grid(64, 64, 64, wl.dt, order=2)
    bn = fields.copy()
    oracle.half_b(g, bn)
    rng = np.random.Generator(np.random.PCG64(98))
    for p in rng.choice(e.n, 3000, replace=False):
        E, B = oracle.gather(g, bn, x0[:, p])
        wn = oracle.push(-1.0, wl.dt, 1.0, E, B, w0[:, p])
        xn = x0[:, p] + oracle.displacement(g, wn)
        assert np.max(np.abs(wn - w1[:, p])) <= 1e-12 * max(1e-3, np.max(np.abs(wn)))
        assert np.max(np.abs(_wrapdiff(xn, x1[:, p], 64))) <= 1e-12 * 64
    d = sim.diagnostics()
    assert d["gauss_rel"] <= 1e-12, d
    assert d["nonfinite"] == 0
    sim.close()


def test_order2_rejected_where_not_built():
    from paper_1101_0809_amd import Sim
    from paper_1101_0809_amd._lib import PicError
    with pytest.raises(PicError):
        Sim(nx=8, ny=8, nz=1, dt=0.5, dims=2, precision="fp32c", order=2)
    with pytest.raises(PicError):
        Sim(nx=8, ny=8, nz=1, dt=0.5, dims=2, order=3)
    import torch
    sim = _sim(nx=8, ny=8, nz=1, dt=0.5, dims=2)
    lam = torch.zeros(6 * 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(PicError):
        sim.adjoint_seed_field_energy(lam)
    sim.close()
