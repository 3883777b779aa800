"""Pins of the oracle's open x boundary (xbc = 1).

The paper's tests are periodic boxes; the open boundary is an extension
around its field update: Mur's first-order absorbing condition on the
tangential B at the walls x = 0 and x = nx - 1, and particles absorbed
(weight set to zero) when a step ends within oracle.ABSORB cells of a wall.
Each test checks the oracle against something other than itself:
- the discrete reflection coefficient of Mur's condition on the staggered
  grid, derived in closed form from the grid's dispersion relation;
- exact transmission at the one-dimensional magic time step c dt = dx;
- the symmetry of Maxwell's equations under a quarter turn about x, which
  ties the B^y walls to the B^z walls;
- the outside layer, which must hold nothing and pass nothing on;
- free streaming, where every particle's absorption step is known in
  closed form;
- the charge-conservation invariant of Section 2 away from the walls, and
  the charge bookkeeping of the absorbed particles.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import picgen

RNG = np.random.Generator(np.random.PCG64(20110108))


def mur_reflection(omega, dt, dx, c=1.0):
    """Reflection coefficient of a plane wave of frequency omega hitting the
    wall at normal incidence.  On the staggered grid a wave uniform in y and z
    obeys sin(omega dt / 2) / (c dt) = sin(kappa dx / 2) / dx.  Write the wall
    field as incident plus r times reflected, B_i^n = z^n (p^-i + r p^i) with
    z = exp(i omega dt), p = exp(i kappa dx), wall at i = 0 and the plane one
    cell inside at i = -1.  Mur's update
    B_0^{n+1} = B_{-1}^n + k (B_{-1}^{n+1} - B_0^n), k = (c dt - dx)/(c dt + dx),
    then gives z (1 + r) = (p + r/p) + k (z (p + r/p) - (1 + r)), solved for r."""
    kappa = 2.0 * math.asin(dx * math.sin(omega * dt / 2.0) / (c * dt)) / dx
    z, p = cmath.exp(1j * omega * dt), cmath.exp(1j * kappa * dx)
    k = (c * dt - dx) / (c * dt + dx)
    return -(z - p - k * (z * p - 1.0)) / (z - 1.0 / p - k * (z / p - 1.0))


def _amplitude(y, t, omega):
    """Amplitude of the sinusoid of frequency omega fitted to samples y(t)."""
    A = np.stack([np.cos(omega * t), np.sin(omega * t)], axis=1)
    co, *_ = np.linalg.lstsq(A, np.asarray(y), rcond=None)
    return math.hypot(*co), np.max(np.abs(np.asarray(y) - A @ co))


@pytest.mark.parametrize("wavelength,dt", [(16, 0.5), (8, 0.5), (12, 0.3)])
def test_mur_reflection_matches_the_discrete_closed_form(wavelength, dt):
    """The plane-wave source sends E^y along +x to the right wall.  Left of the
    source plane only the reflected wave is present (the total-field /
    scattered-field plane leaks nothing in vacuum), so in steady state the
    ratio of its amplitude to the incident one (read on the source's own
    auxiliary line) is |r|.  The reflected wave reflects once more at the
    left wall, which perturbs the measurement at order |r|^2."""
    nx, plane = 200, 60
    omega = 2 * math.pi / wavelength
    steps_per_period = round(2 * math.pi / omega / dt)
    assert abs(steps_per_period * dt * omega - 2 * math.pi) < 1e-12
    st = oracle.State(oracle.Grid(nx, 2, 1, dt, source=(plane, 1.0, omega, 8 * math.pi / omega), xbc=1), [])
    n0 = int(2 * (4 * 2 * math.pi / omega + 2 * nx) / dt)  # ramp plus two crossings of the box
    st.step(n0)
    probe, aux_probe = 30, 20
    nwin = 10 * steps_per_period
    rec, inc = np.empty(nwin), np.empty(nwin)
    for n in range(nwin):
        st.step(1)
        rec[n] = st.fields[1][0, 0, probe]
        inc[n] = st.aux[aux_probe]
    t = (n0 + 1 + np.arange(nwin)) * dt
    a_inc, res_inc = _amplitude(inc, t, omega)
    a_ref, _ = _amplitude(rec, t, omega)
    assert res_inc < 1e-3 * a_inc            # the incident wave is steady
    r = abs(mur_reflection(omega, dt, 1.0))
    assert 1e-3 < r < 0.1
    assert abs(a_ref / a_inc - r) < 2.0 * r * r + 1e-6, (a_ref / a_inc, r)


def test_mur_is_exact_at_the_magic_time_step():
    """In one dimension at c dt = dx the staggered scheme moves each half of a
    pulse by one cell per step without error, and Mur's condition (k = 0)
    copies the inside value to the wall: both halves of an E^y pulse and of
    an E^z pulse leave through the two walls without any reflection.  A
    periodic box keeps the energy."""
    nx = 120
    x = np.arange(nx) + 0.5
    energies = {}
    for xbc in (0, 1):
        st = oracle.State(oracle.Grid(nx, 1, 1, 1.0, xbc=xbc), [])
        st.fields[1][0, 0, :] = np.exp(-((x - 60.0) / 6.0) ** 2)
        st.fields[2][0, 0, :] = np.exp(-((x - 45.0) / 4.0) ** 2)
        st.fields[1:3, 0, 0, nx - 1] = 0.0
        e0 = np.sum(st.fields[:6] ** 2)
        st.step(110)
        energies[xbc] = np.sum(st.fields[:6] ** 2) / e0
    assert energies[1] < 1e-30
    assert energies[0] > 0.99


def test_both_polarisations_are_absorbed_alike():
    """Maxwell's equations are symmetric under a quarter turn about x, which
    takes (E^y, B^z) to (E^z, -B^y).  A wave uniform in y and z sees the same
    grid either way, so an E^z pulse must evolve, through both walls, as the
    E^y pulse turned: E^z = E^y and B^y = -B^z at every step."""
    nx, dt = 80, 0.5
    x = np.arange(nx) + 0.5
    prof = np.exp(-((x - 30.0) / 3.0) ** 2) * np.cos(0.9 * x)
    prof[nx - 1] = 0.0
    a = oracle.State(oracle.Grid(nx, 1, 1, dt, xbc=1), [])
    b = oracle.State(oracle.Grid(nx, 1, 1, dt, xbc=1), [])
    a.fields[1][0, 0, :] = prof
    b.fields[2][0, 0, :] = prof
    for _ in range(6):
        a.step(25)
        b.step(25)
        assert np.array_equal(b.fields[2], a.fields[1])
        assert np.array_equal(b.fields[4], -a.fields[5])
    assert np.max(np.abs(a.fields[1])) < 0.05   # most of it has left


def test_pulse_leaves_the_box_in_three_dimensions():
    """A localised E^y pulse in a 3D box, at a Courant number below the
    magic one, splits into waves that leave through the walls; what stays
    is of the order |r|^2 of the energy that hit them."""
    nx, ny, nz, dt = 64, 4, 4, 0.45
    x = np.arange(nx) + 0.5
    st = oracle.State(oracle.Grid(nx, ny, nz, dt, xbc=1), [])
    st.fields[1][:, :, :] = np.exp(-((x - 32.0) / 5.0) ** 2)
    st.fields[1][:, :, nx - 1] = 0.0
    e0 = np.sum(st.fields[:6] ** 2)
    st.step(200)
    assert np.sum(st.fields[:6] ** 2) / e0 < 1e-4


def test_outside_layer_carries_nothing():
    """The cell layer x in [nx - 1, nx) lies outside the box: whatever it
    holds at the start, after a step its E^y, E^z and B^x are zero and the
    fields inside the box are those of a run that started with it empty."""
    nx, ny, nz = 20, 5, 4
    base = RNG.normal(0.0, 1.0, (9, nz, ny, nx))
    base[6:] = 0.0
    base[1:4, :, :, nx - 1] = 0.0
    noisy = base.copy()
    noisy[1:4, :, :, nx - 1] = RNG.normal(0.0, 1.0, (3, nz, ny))
    runs = []
    for f in (base, noisy):
        st = oracle.State(oracle.Grid(nx, ny, nz, 0.4, xbc=1), [], fields=f)
        st.step(3)
        runs.append(st.fields)
        assert np.all(st.fields[1:4, :, :, nx - 1] == 0.0)
    inside = (slice(0, 6), slice(None), slice(None), slice(0, nx - 1))
    assert np.array_equal(runs[0][inside], runs[1][inside])
    assert np.array_equal(runs[0][0:6, :, :, nx - 1][[0, 4, 5]], runs[1][0:6, :, :, nx - 1][[0, 4, 5]])


def test_free_streaming_particles_are_absorbed_at_the_predicted_step():
    """Without charge no field arises and each particle moves by the constant
    (u_x / c) c dt / dx per step (Appendix, Eq. coordscheme).  It is absorbed
    after the first step that ends at x < ABSORB or x >= nx - 1 - ABSORB, and
    keeps its weight until then."""
    nx, dt, n, nsteps = 32, 0.5, 400, 40
    L = oracle.ABSORB
    x = np.stack([RNG.uniform(L + 0.01, nx - 1 - L - 0.01, n), RNG.uniform(0, 4, n), RNG.uniform(0, 4, n)])
    w = RNG.normal(0.0, 0.4, (3, n))
    sp = oracle.Species(x, w, np.full(n, 0.5), q=0.0, m=1.0)
    st = oracle.State(oracle.Grid(nx, 4, 4, dt, xbc=1), [sp])
    vx = w[0] / np.sqrt(1.0 + np.sum(w * w, axis=0)) * dt
    steps = np.arange(1, nsteps + 1)[:, None]
    path = x[0][None, :] + steps * vx[None, :]
    out = (path < L) | (path >= nx - 1 - L)
    expected = np.where(out.any(axis=0), np.argmax(out, axis=0) + 1, nsteps + 1)
    near = np.min(np.minimum(np.abs(path - L), np.abs(path - (nx - 1 - L))), axis=0) < 1e-9
    seen = np.full(n, nsteps + 1)
    for s in range(1, nsteps + 1):
        st.step(1)
        gone = (sp.weight == 0.0) & (seen > nsteps)
        seen[gone] = s
    assert np.all(sp.weight[seen > nsteps] == 0.5)
    assert np.array_equal(seen[~near], expected[~near])
    assert 50 < np.count_nonzero(expected <= nsteps) < n - 50


def test_open_x_plasma_keeps_gauss_inside_and_loses_only_absorbed_charge():
    """Two counter-streaming electron beams on an immobile ion background run
    into both walls.  The current deposit conserves charge, so R = div E -
    4 pi rho keeps its initial value wherever no absorbed particle's charge
    support reaches: cells ABSORB + 1 .. nx - 3 - ABSORB.  div B keeps its
    value at the nodes whose B all follow the curl of E: 1 .. nx - 2.  The
    total charge drops by exactly the absorbed particles' charge."""
    wl = picgen.Workload("open", 24, 6, 6, 3, 0.45, 3, (0.05,) * 3, 0.3, 24, drift=0.5)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    g = oracle.Grid(24, 6, 6, wl.dt, xbc=1)
    ions = oracle.Species(ion.x, ion.w, ion.weight, q=1.0, m=100.0, mobile=False)
    el = oracle.Species(e.x, e.w, e.weight)
    st = oracle.State(g, [el, ions])
    L = oracle.ABSORB
    inner = slice(L + 1, g.nx - 2 - L)
    R0 = st.gauss_residual()
    D0 = st.div_b()
    V = g.dx * g.dy * g.dz
    q0 = V * np.sum(st.rho())
    w0 = el.weight.copy()
    rho_e = np.max(np.abs(4 * np.pi * st.rho([el])))
    st.step(wl.steps)
    dR = st.gauss_residual() - R0
    assert np.max(np.abs(dR[:, :, inner])) / rho_e < 1e-12
    absorbed = w0 - el.weight
    assert np.count_nonzero(absorbed) > 50
    assert np.all((el.weight == 0) | (el.weight == w0))
    assert V * np.sum(st.rho()) == pytest.approx(q0 - el.q * np.sum(absorbed), abs=1e-12 * abs(q0) + 1e-12)
    assert np.max(np.abs(dR[:, :, :])) / rho_e > 1e-3       # absorption does leave its mark near the walls
    assert np.max(np.abs((st.div_b() - D0)[:, :, 1:g.nx - 1])) < 1e-13
