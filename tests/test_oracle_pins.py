"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numerical
integration of the definitions, exact identities stated in the paper, closed
forms (gyration, cold plasma oscillation, vacuum dispersion, self-force) or
values printed in the paper (tests/golden/paper_values.json).  Section and
equation names refer to arXiv:1101.0809.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import picgen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
RNG = np.random.Generator(np.random.PCG64(20110105))


# --------------------------------------------------------------------------
# Q1  form factors (Section 3.1, Section 4.5)
# --------------------------------------------------------------------------

def _cap(r):
    return 1.0 if abs(r) <= 0.5 else 0.0


@pytest.mark.parametrize("l", [1, 2, 3])
def test_form_factor_is_recursive_integral(l):
    """f^(l)(r) equals the integral of f^(l-1) over [r-1/2, r+1/2] (Section 3.1);
    the order-0 base is the unit cap."""
    lower = _cap if l == 1 else (lambda t: oracle.shape(l - 1, t))
    knots = [k * 0.5 for k in range(-6, 7)]
    for r in np.concatenate([RNG.uniform(-2.5, 2.5, 40), [0.0, 0.5, 1.0, 1.5, -0.25]]):
        pts = [p for p in knots if r - 0.5 < p < r + 0.5]
        ref, _ = integrate.quad(lower, r - 0.5, r + 0.5, points=pts or None, epsabs=1e-14,
                                epsrel=1e-13)
        assert oracle.shape(l, r) == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_form_factor_symmetry_support_partition(l):
    """Symmetric in r, zero for |r| > (l+1)/2, and sum_i f(x+i) = 1 (Eq. sum1)."""
    for r in RNG.uniform(0, 3, 30):
        assert oracle.shape(l, r) == oracle.shape(l, -r)
        if r > (l + 1) / 2:
            assert oracle.shape(l, r) == 0.0
    for x in RNG.uniform(-0.5, 0.5, 30):
        s = sum(oracle.shape(l, x + i) for i in range(-4, 5))
        assert s == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_form_factor_derivative_identity(l):
    """d f^(l)/dr = f^(l-1)(r + 1/2) - f^(l-1)(r - 1/2) (Section 3.1, property 3)."""
    lower = _cap if l == 1 else (lambda t: oracle.shape(l - 1, t))
    h = 1e-7
    for r in RNG.uniform(-2.2, 2.2, 30):
        if min(abs(r - k * 0.5) for k in range(-6, 7)) < 1e-4:
            continue
        fd = (oracle.shape(l, r + h) - oracle.shape(l, r - h)) / (2 * h)
        assert fd == pytest.approx(lower(r + 0.5) - lower(r - 0.5), abs=1e-6)


def test_cumulative_is_integral_of_hat():
    """F_i(x_p) = integral of f^(1) up to the node (Section 3.1)."""
    for s in np.concatenate([RNG.uniform(-1.5, 1.5, 40), [-1.0, 0.0, 1.0]]):
        ref, _ = integrate.quad(lambda t: oracle.shape(1, t), -2.0, s, points=[-1, 0, 1],
                                epsabs=1e-14)
        assert oracle.cumulative1(s) == pytest.approx(ref, abs=1e-13)


def test_cumulative2_is_integral_of_quadratic():
    """The order-2 cumulative form factor is the integral of f^(2) (Section
    3.1 one order up), for the current of the order-2 1/2 scheme."""
    for s in np.concatenate([RNG.uniform(-2.0, 2.0, 40), [-1.5, -0.5, 0.0, 0.5, 1.5]]):
        ref, _ = integrate.quad(lambda t: oracle.shape(2, t), -2.0, s, points=[-1.5, -0.5, 0.5, 1.5],
                                epsabs=1e-14)
        assert oracle.cumulative2(s) == pytest.approx(ref, abs=1e-13)


def test_alternating_order_table_1p5():
    """Oracle point and cell weights equal the printed order-1 1/2 table (Section 4.5)."""
    for xp in RNG.uniform(0, 10, 40):
        i = math.floor(xp)
        d = xp - i
        assert oracle.shape(1, i - xp) == pytest.approx(1 - d, abs=1e-15)
        assert oracle.shape(1, i + 1 - xp) == pytest.approx(d, abs=1e-15)
        table = [(1 - d) ** 2 / 2, 0.75 - (0.5 - d) ** 2, d ** 2 / 2]
        for o, ref in zip((-1, 0, 1), table):
            assert oracle.shape(2, (i + o) + 0.5 - xp) == pytest.approx(ref, abs=1e-15)


def test_alternating_order_table_2p5():
    """The order-2 1/2 table of Section 4.5 equals f^(2) at nodes and f^(3) at
    cell centres (the oracle's shape functions one order up)."""
    for xp in RNG.uniform(0, 10, 40):
        i = math.floor(xp + 0.5)
        d = xp + 0.5 - i
        fnode = [(1 - d) ** 2 / 2, 0.75 - (0.5 - d) ** 2, d ** 2 / 2]
        for o, ref in zip((-1, 0, 1), fnode):
            assert oracle.shape(2, (i + o) - xp) == pytest.approx(ref, abs=1e-14)
        fcell = [(1 - d) ** 3 / 6, (2 - d) ** 3 / 6 - 2 * (1 - d) ** 3 / 3,
                 (1 + d) ** 3 / 6 - 2 * d ** 3 / 3, d ** 3 / 6]
        for o, ref in zip((-2, -1, 0, 1), fcell):
            assert oracle.shape(3, (i + o) + 0.5 - xp) == pytest.approx(ref, abs=1e-14)


# --------------------------------------------------------------------------
# Q2-Q4  current and charge (Section 3.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("order", [1, 2])
def test_cumulative_sum_identity(order):
    """sum_i [F_i(x) - F_i(x')] = x' - x (Eq. sumcurrent), for the cumulative
    of f^(1) and of f^(2)."""
    F = oracle.cumulative1 if order == 1 else oracle.cumulative2
    for _ in range(30):
        x = RNG.uniform(3, 7)
        xq = x + RNG.uniform(-1.5, 1.5)
        s = sum(F(i - x) - F(i - xq) for i in range(-2, 14))
        assert s == pytest.approx(xq - x, abs=1e-14)


def _grid(n=8, dt=0.4, **kw):
    return oracle.Grid(n, n, n, dt, **kw)


@pytest.mark.parametrize("order", [1, 2])
def test_face_sum_equals_velocity(order):
    """sum over faces of xi^x equals u^x (Section 3.2, exact relationship)."""
    g = _grid(10, dt=0.37, dx=1.3, dy=0.8, dz=1.1, order=order)
    V = g.dx * g.dy * g.dz
    for _ in range(20):
        x0 = RNG.uniform(2, 8, 3)
        x1 = x0 + RNG.uniform(-0.95, 0.95, 3)
        J = oracle.deposit(g, x0, x1, charge=1.0)
        h = np.array([g.dx, g.dy, g.dz])
        u = (x1 - x0) * h / g.dt
        for a in range(3):
            assert J[a].sum() * V == pytest.approx(u[a], abs=1e-14)


def _box_path_current(x0, x1, n, dt, h, order=1):
    """Mean over the six axis orderings of the box-path integrals of Eq. Jx
    (Section 3.2).  F_i and Delta F are obtained by numerical integration of the
    node form factor f^(order) (their definitions, Eq. intff), not from closed
    forms: the hat for order 1, the quadratic spline (the hat integrated over
    a unit cell, done numerically here too) for order 2."""
    hat = lambda t: max(0.0, 1.0 - abs(t))
    if order == 1:
        f, knots = hat, (-1.0, 0.0, 1.0)
    else:
        f = lambda t: integrate.quad(hat, t - 0.5, t + 0.5, points=[-1.0, 0.0, 1.0], epsabs=1e-15)[0]
        knots = (-1.5, -0.5, 0.5, 1.5)

    def F(i, xp):  # cumulative form factor at node i
        lo = min(i, xp - 2.0)
        return integrate.quad(lambda t: f(t - xp), lo - 1.0, i,
                              points=[xp + k for k in knots], epsabs=1e-15, limit=200)[0]

    def dF(c, xp):  # integral over the cell [c, c+1]
        return integrate.quad(lambda t: f(t - xp), c, c + 1, points=[xp + k for k in knots],
                              epsabs=1e-15, limit=200)[0]

    import itertools
    J = np.zeros((3, n, n, n))
    lo = np.floor(np.minimum(x0, x1)).astype(int) - 2
    hi = np.floor(np.maximum(x0, x1)).astype(int) + 3
    for order in itertools.permutations(range(3)):
        p = np.array(x0, dtype=float)
        for axis in order:
            q = p.copy()
            q[axis] = x1[axis]
            t1, t2 = (axis + 1) % 3, (axis + 2) % 3
            for a in range(lo[axis], hi[axis] + 1):
                dfa = F(a, q[axis]) - F(a, p[axis])
                if dfa == 0.0:
                    continue
                for b in range(lo[t1], hi[t1] + 1):
                    for c in range(lo[t2], hi[t2] + 1):
                        ijk = [0, 0, 0]
                        ijk[axis], ijk[t1], ijk[t2] = a % n, b % n, c % n
                        J[axis][ijk[2], ijk[1], ijk[0]] += (
                            -(h[axis] / dt) * dfa * dF(b, p[t1]) * dF(c, p[t2]) / 6.0)
            p = q
    return J


@pytest.mark.parametrize("order", [1, 2])
def test_current_equals_six_box_path_average(order):
    """The one-sixth and one-quarter forms of Eq. current both equal the mean of
    the six box-path integrals, computed here from the definitions."""
    n, dt = 8, 0.45
    h = np.array([1.0, 1.0, 1.0])
    g = oracle.Grid(n, n, n, dt, order=order)
    cases = [(np.array([3.3, 3.7, 4.1]), np.array([3.9, 4.2, 3.6])),
             (np.array([4.05, 3.5, 3.95]), np.array([3.4, 3.5, 4.4])),
             (np.array([3.5, 3.5, 3.5]), np.array([3.5, 3.5, 3.5]) + 0.2)]
    if order == 2:
        cases = cases[:2]  # nested quadrature: keep the run short
    for x0, x1 in cases:
        ref = _box_path_current(x0, x1, n, dt, h, order)
        six = oracle.deposit(g, x0, x1, charge=1.0, form="sixth")
        quarter = oracle.deposit(g, x0, x1, charge=1.0, form="quarter")
        assert np.max(np.abs(six - ref)) < 1e-12
        assert np.max(np.abs(quarter - ref)) < 1e-12


def _div_face(g, J):
    return ((np.roll(J[0], -1, axis=2) - J[0]) / g.dx + (np.roll(J[1], -1, axis=1) - J[1]) / g.dy
            + (np.roll(J[2], -1, axis=0) - J[2]) / g.dz)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("form", ["sixth", "quarter"])
def test_single_particle_continuity(form, order):
    """(rho^{n+1} - rho^n)/dt + div J = 0 for one particle, any move of less
    than a cell, including moves across the periodic boundary (Eq. chargelaw)."""
    g = oracle.Grid(7, 6, 5, 0.41, dx=1.2, dy=0.9, dz=1.05, order=order)
    x0s, x1s = picgen.random_moves(60, seed=7, box=(7, 6, 5), max_step=0.95)
    for p in range(x0s.shape[1]):
        x0, x1 = x0s[:, p], x1s[:, p]
        q = 0.7
        J = oracle.deposit(g, x0, x1, charge=q, form=form)
        r0 = oracle.rho_of(g, x0, q)
        r1 = oracle.rho_of(g, x1 % np.array([7, 6, 5]), q)
        resid = (r1 - r0) / g.dt + _div_face(g, J)
        assert np.max(np.abs(resid)) < 1e-13 * max(1.0, np.max(np.abs(r0)) / g.dt)


# --------------------------------------------------------------------------
# Q5  whole-run Gauss law and div B invariants (Section 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (1.0, 0.8, 1.25)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("shape", [(6, 5, 4), (8, 8, 1)])
def test_gauss_and_divb_invariant(shape, order, cell):
    """Unequal cell sizes make every curl coefficient and divergence term
    carry its own axis's size."""
    nx, ny, nz = shape
    wl = picgen.Workload("pin", nx, ny, nz, 3 if nz > 1 else 2, 0.45, 4, (0.2,) * 3, 0.3, 20)
    e = picgen.electrons(wl)
    ions = picgen.ions_like(wl, e)
    dx, dy, dz = cell
    st = oracle.State(oracle.Grid(nx, ny, nz, wl.dt, dx=dx, dy=dy, dz=dz, order=order),
                      [oracle.Species(e.x, e.w, e.weight, q=-1.0, m=1.0),
                       oracle.Species(ions.x, ions.w, ions.weight, q=1.0, m=100.0, mobile=False)])
    # start from a non-trivial field with zero divergence of B
    st.fields[0:3] = RNG.normal(0, 1e-3, (3,) + st.grid.shape)
    R0 = st.gauss_residual()
    D0 = st.div_b()
    rho_e0 = np.max(np.abs(4 * np.pi * st.rho(st.species[:1])))
    st.step(20)
    R = st.gauss_residual()
    assert np.max(np.abs(R - R0)) / rho_e0 < 1e-12
    assert np.max(np.abs(st.div_b() - D0)) < 1e-14
    # positions stay in the box
    for a, n in enumerate(shape):
        assert np.all((st.species[0].x[a] >= 0) & (st.species[0].x[a] < n))


def test_free_streaming_displacement():
    """Eq. coordscheme on unequal cells: in zero field a particle advances
    (w_a / gamma) c dt / h_a cells per step along axis a, with
    gamma = sqrt(1 + w^2 / c^2).  The weights are so small that the
    particles' own fields do not move them measurably."""
    dx, dy, dz, dt = 1.0, 0.8, 1.25, 0.45
    nx, ny, nz = 16, 20, 12
    w = np.array([[0.3, -1.2, 2.5], [0.0, 0.7, -0.4], [-0.9, 0.05, 1.5]])
    x0 = np.array([[3.2, 7.5, 12.9], [4.4, 10.1, 0.3], [6.7, 2.2, 9.8]])
    st = oracle.State(oracle.Grid(nx, ny, nz, dt, dx=dx, dy=dy, dz=dz),
                      [oracle.Species(x0.copy(), w.copy(), np.full(3, 1e-14), q=-1.0, m=1.0)])
    n = 10
    st.step(n)
    gam = np.sqrt(1.0 + np.sum(w ** 2, axis=0))
    for a, (h, L) in enumerate(((dx, nx), (dy, ny), (dz, nz))):
        expect = np.mod(x0[a] + n * (w[a] / gam) * dt / h, L)
        diff = (st.species[0].x[a] - expect + L / 2) % L - L / 2
        assert np.max(np.abs(diff)) < 1e-9, (a, diff)


# --------------------------------------------------------------------------
# Q6  push: magnetic energy neutrality (Eq. p2), pure electric kick, partition
# --------------------------------------------------------------------------

def test_push_magnetic_neutrality():
    for _ in range(50):
        E = RNG.normal(0, 1, 3)
        B = RNG.normal(0, 3, 3)
        w = RNG.normal(0, 2, 3)
        qm, dt, c = RNG.choice([-1.0, 1.0, 0.01]), 0.3, 1.0
        w1 = oracle.push(qm, dt, c, E, B, w)
        e = 0.5 * qm * dt * E
        lhs = np.sum((w1 - e) ** 2)
        rhs = np.sum((w + e) ** 2)
        assert lhs == pytest.approx(rhs, rel=2e-15)


def test_push_pure_electric_kick():
    for _ in range(20):
        E = RNG.normal(0, 1, 3)
        w = RNG.normal(0, 1, 3)
        w1 = oracle.push(-1.0, 0.25, 1.0, E, np.zeros(3), w)
        assert np.allclose(w1, w - 0.25 * E, rtol=0, atol=1e-15)


@pytest.mark.parametrize("qm", [-1.0, 1.0])
def test_push_rotation_sense(qm):
    """Eq. (1): dw/dt = (q/m)(E + u/c x B).  In a pure magnetic field along +z
    the Appendix's rotation turns w by theta = 2 atan(|q/m| (dt/2) B / gamma)
    about +z when q < 0 (counter-clockwise) and about -z when q > 0: the
    exact image of w = (w0, 0, 0) is w0 (cos theta, -sign(q) sin theta, 0).
    Swapping the order of a cross product in the push reverses the turn."""
    dt, c, b, w0 = 0.3, 1.0, 0.7, 0.6
    gam = math.sqrt(1.0 + w0 * w0)
    theta = 2.0 * math.atan(abs(qm) * 0.5 * dt * b / gam)
    w1 = oracle.push(qm, dt, c, np.zeros(3), np.array([0.0, 0.0, b]), np.array([w0, 0.0, 0.0]))
    ref = w0 * np.array([math.cos(theta), -math.copysign(1.0, qm) * math.sin(theta), 0.0])
    assert np.allclose(w1, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("order,interp", [(1, 0), (2, 0), (1, 1)])
def test_gather_partition_of_unity(order, interp):
    """Uniform grid fields are reproduced exactly at any position (Eq. one),
    for both alternating orders and for the conventional interpolation."""
    g = oracle.Grid(5, 4, 6, 0.3, order=order, interp=interp)
    vals = RNG.normal(0, 1, 6)
    fields = np.zeros((9,) + g.shape)
    for c in range(6):
        fields[c] = vals[c]
    for _ in range(20):
        xp = RNG.uniform(0, 1, 3) * np.array([5, 4, 6])
        E, B = oracle.gather(g, fields, xp)
        assert np.allclose(np.concatenate([E, B]), vals, atol=1e-14, rtol=0)


def test_gather_stencil_order2_matches_table():
    """Order 2 1/2: a unit value at one grid point of each component comes
    back at the particle as the product of the printed Section 4.5 table
    entries: node factors f_{i-1:i+1} along the component's own axis for E
    (along the other two for B), cell factors Delta F_{i-3/2:i+3/2} on the
    rest, with i = int(x_p + 1/2) per axis."""
    n = 9
    g = oracle.Grid(n, n, n, 0.3, order=2)

    def table(x):
        i = math.floor(x + 0.5)
        d = x + 0.5 - i
        node = {i - 1: (1 - d) ** 2 / 2, i: 0.75 - (0.5 - d) ** 2, i + 1: d ** 2 / 2}
        cell = {i - 2: (1 - d) ** 3 / 6, i - 1: (2 - d) ** 3 / 6 - 2 * (1 - d) ** 3 / 3,
                i: (1 + d) ** 3 / 6 - 2 * d ** 3 / 3, i + 1: d ** 3 / 6}
        return node, cell
    node_axes = {0: (0,), 1: (1,), 2: (2,), 3: (1, 2), 4: (0, 2), 5: (0, 1)}
    for _ in range(6):
        xp = RNG.uniform(3, 6, 3)
        tabs = [table(xp[a]) for a in range(3)]
        for comp in range(6):
            for _ in range(4):
                pt = [int(RNG.integers(math.floor(xp[a]) - 2, math.floor(xp[a]) + 3)) for a in range(3)]
                fields = np.zeros((9, n, n, n))
                fields[comp][pt[2] % n, pt[1] % n, pt[0] % n] = 1.0
                E, B = oracle.gather(g, fields, xp)
                got = np.concatenate([E, B])[comp]
                ref = 1.0
                for a in range(3):
                    node, cell = tabs[a]
                    ref *= (node if a in node_axes[comp] else cell).get(pt[a], 0.0)
                assert got == pytest.approx(ref, abs=1e-15)


def test_conventional_gather_matches_eq_wrong1():
    """The conventional interpolation (Eq. wrong1 and its analogue for B): a
    unit value at one grid point comes back as the mean of the two adjacent
    cell factors along each node axis of the component times the cell factor
    along the others, with the printed order-1 1/2 cell factors (Section 4.5)."""
    n = 9
    g = oracle.Grid(n, n, n, 0.3, interp=1)

    def cellf(x):
        i = math.floor(x)
        d = x - i
        return {i - 1: (1 - d) ** 2 / 2, i: 0.75 - (0.5 - d) ** 2, i + 1: d ** 2 / 2}
    node_axes = {0: (0,), 1: (1,), 2: (2,), 3: (1, 2), 4: (0, 2), 5: (0, 1)}
    for _ in range(6):
        xp = RNG.uniform(3, 6, 3)
        cf = [cellf(xp[a]) for a in range(3)]
        for comp in range(6):
            for _ in range(4):
                pt = [int(RNG.integers(math.floor(xp[a]) - 2, math.floor(xp[a]) + 3)) for a in range(3)]
                fields = np.zeros((9, n, n, n))
                fields[comp][pt[2], pt[1], pt[0]] = 1.0
                E, B = oracle.gather(g, fields, xp)
                ref = 1.0
                for a in range(3):
                    if a in node_axes[comp]:
                        ref *= 0.5 * (cf[a].get(pt[a] - 1, 0.0) + cf[a].get(pt[a], 0.0))
                    else:
                        ref *= cf[a].get(pt[a], 0.0)
                assert np.concatenate([E, B])[comp] == pytest.approx(ref, abs=1e-15)


def test_conventional_interpolation_conserves_charge_but_not_energy():
    """Section 5, Fig. 2: with the conventional interpolation the Gauss
    invariant still holds (the current is the same), but the total-energy
    defect of a thermal plasma (v_Te = 0.05 c, 2 electrons per cell, mesh =
    Debye length, c dt = dx / 2, co-located ions) is far larger than with the
    alternating-order form factor: the paper reports two orders of magnitude.
    Measured here on 12^3 cells over 60 steps: about 1e-5 against 5e-3."""
    n = 12
    wl = picgen.Workload("x1", n, n, n, 3, 0.5, 2, (0.05,) * 3, 0.05, 60, seed=7)
    e = picgen.electrons(wl)
    ions = picgen.ions_like(wl, e)
    defects = []
    for interp in (0, 1):
        st = oracle.State(oracle.Grid(n, n, n, wl.dt, interp=interp),
                          [oracle.Species(e.x.copy(), e.w.copy(), e.weight, q=-1.0, m=1.0),
                           oracle.Species(ions.x, ions.w, ions.weight, q=1.0, m=100.0, mobile=False)])
        R0 = st.gauss_residual()
        rho_e0 = np.max(np.abs(4 * np.pi * st.rho(st.species[:1])))
        tot0 = st.energies().sum()
        st.step(wl.steps)
        assert np.max(np.abs(st.gauss_residual() - R0)) / rho_e0 < 1e-12
        defects.append(abs(st.energies().sum() - tot0) / tot0)
    assert defects[0] < 1e-4
    assert defects[1] > 30 * defects[0], defects


@pytest.mark.parametrize("dx", [1.0, 1.25])
def test_field_energies_of_one_mode(dx):
    """The field energies (Section 4.1) of one Fourier mode, in closed form.
    E^y = A sin(2 pi m i / nx), uniform in y and z, and B^{n-1/2} = 0.  The
    magnetic energy is taken at B^n, the stored B^{n-1/2} advanced half a step
    by Eq. updateB: B^z = -(c dt / dx) A sin(pi m / nx) cos(2 pi m (i + s) / nx)
    for a fixed stagger s, and B^x = B^y = 0.  Over the N cells of volume V,
    V/(8 pi) sum (E^y)^2 = V/(8 pi) A^2 N / 2, and
    V/(8 pi) sum (B^z)^2 = V/(8 pi) (c dt / dx)^2 A^2 sin^2(pi m / nx) N / 2."""
    nx, ny, nz, m, A, dt = 16, 4, 3, 3, 0.7, 0.45
    dy, dz = 0.8, 1.1
    st = oracle.State(oracle.Grid(nx, ny, nz, dt, dx=dx, dy=dy, dz=dz), [])
    st.fields[1] = A * np.sin(2 * np.pi * m * np.arange(nx) / nx)[None, None, :]
    kin, half, fe, fb = st.energies()
    V, N = dx * dy * dz, nx * ny * nz
    assert kin == 0.0 and half == 0.0
    assert fe == pytest.approx(V / (8 * np.pi) * A ** 2 * N / 2, rel=1e-13)
    assert fb == pytest.approx(V / (8 * np.pi) * (dt / dx) ** 2 * A ** 2 * np.sin(np.pi * m / nx) ** 2 * N / 2,
                               rel=1e-12)


def test_half_step_energy_term_is_half_the_work_of_a_step():
    """Section 4.1: the particle energy at t^n is K^{n-1/2} plus the half-step
    term H^n = sum (q dt / 2) u^{n-1/2} . E(x^n).  Over the step that follows,
    E^n does the work K^{n+1/2} - K^{n-1/2} = sum q dt u^n . E(x^n) (the
    magnetic rotation does none), so H^n equals half of it up to O(dt^2)
    terms.  A coherent Langmuir oscillation (Section 5: one electron per cell
    of doubled charge, all drifting at 0.1 c, co-located ions, 8^3 cells)
    moves energy between particles and field within each step; the term must
    follow that exchange in sign and size, and with it the total energy is
    conserved far better than without it.  A sign error in H fails both."""
    n, dt = 8, 0.5
    wl = picgen.Workload("langmuir", n, n, n, 3, dt, 1, (0.0,) * 3, 0.05, 120, seed=31)
    e = picgen.electrons(wl)
    e.w[0] += 0.1
    weight = 2.0 * e.weight
    st = oracle.State(oracle.Grid(n, n, n, dt),
                      [oracle.Species(e.x, e.w, weight, q=-1.0, m=1.0),
                       oracle.Species(e.x, np.zeros_like(e.w), weight, q=1.0, m=100.0, mobile=False)])
    en = [st.energies()]
    for _ in range(wl.steps):
        st.step(1)
        en.append(st.energies())
    en = np.array(en)
    K, H, W = en[:, 0], en[:, 1], en[:, 2] + en[:, 3]
    half_work = 0.5 * (K[1:] - K[:-1])
    assert np.max(W) > 0.2 * K[0]   # the oscillation moves a good part of K into the field
    mismatch = np.sum(np.abs(H[:-1] - half_work)) / np.sum(np.abs(half_work))
    assert mismatch < 0.05, mismatch
    with_term = np.max(np.abs(K + H + W - (K + H + W)[0])) / K[0]
    without = np.max(np.abs(K + W - (K + W)[0])) / K[0]
    assert with_term < 0.05 * without, (with_term, without)


# --------------------------------------------------------------------------
# Q7  closed-form gyration of a test particle (Section 5, gyration test)
# --------------------------------------------------------------------------

def test_gyration_closed_form():
    gy = GOLDEN["gyration"]
    dt = gy["omega_B_dt"] / gy["omega_B"]
    dx = 1.0 * dt / gy["c_dt_over_dx"]
    n = 32
    steps = int(round(gy["omega_B_t_end"] / gy["omega_B_dt"]))
    g = oracle.Grid(n, n, n, dt, dx=dx, dy=dx, dz=dx, bext=(0.0, 0.0, gy["omega_B"]))
    x = np.array([[n / 2], [n / 2], [n / 2]])
    w = np.array([[gy["w_over_c"]], [0.0], [0.0]])
    sp = oracle.Species(x, w, np.ones(1), q=-1.0, m=1.0, deposit=False)
    st = oracle.State(g, [sp])
    gam = math.sqrt(1 + gy["w_over_c"] ** 2)
    theta = 2 * math.atan(gy["omega_B_dt"] / (2 * gam))
    u = gy["w_over_c"] / gam
    R = u * dt / (2 * math.sin(theta / 2)) / dx  # chord geometry, cell units
    pts = [sp.x[:, 0].copy()]
    for _ in range(steps):
        st.step(1)
        pts.append(sp.x[:, 0].copy())
    pts = np.array(pts)
    # the derived numbers quoted for this test
    assert gam == pytest.approx(1.1180340, abs=1e-7)
    assert theta == pytest.approx(0.2226820, abs=1e-7)
    assert R == pytest.approx(1.0062306, abs=1e-7)
    # circumcentre of the first three points; every point must lie on the circle
    a, b, c = pts[0, :2], pts[1, :2], pts[2, :2]
    d = 2 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
    ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
    uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
    r = np.hypot(pts[:, 0] - ux, pts[:, 1] - uy)
    assert np.max(np.abs(r - R)) < 1e-11
    # Eq. (1): dw/dt = (q/m)(u/c x B).  The electron (q < 0) starts along +x in
    # B along +z: u x B points along -y, so the force points along +y and the
    # orbit turns counter-clockwise seen from +z, by +theta per step
    ang = np.unwrap(np.arctan2(pts[:, 1] - uy, pts[:, 0] - ux))
    assert np.allclose(np.diff(ang), theta, atol=1e-11)
    assert np.all(pts[:, 2] == n / 2)
    assert np.sum(sp.w[:, 0] ** 2) == pytest.approx(gy["w_over_c"] ** 2, rel=1e-14)


# --------------------------------------------------------------------------
# Q8  cold k=0 plasma oscillation: leapfrog recurrence
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [2, 3])
def test_cold_plasma_oscillation(dims):
    opdt = GOLDEN["thermal_test"]["omega_pe_dt"]
    nz = 1 if dims == 2 else 4
    wl = picgen.Workload("cold", 4, 4, nz, dims, 0.5, 4 if dims == 2 else 8, (0.0,) * 3,
                         opdt / 0.5, 40)
    e = picgen.lattice_electrons(wl, drift=(1e-5, 0.0, 0.0))
    ions = picgen.Plasma(e.x.copy(), np.zeros_like(e.w), e.weight.copy(), q=1.0, m=1.0)
    st = oracle.State(oracle.Grid(4, 4, nz, wl.dt),
                      [oracle.Species(e.x, e.w, e.weight),
                       oracle.Species(ions.x, ions.w, ions.weight, q=1.0, m=1.0, mobile=False)])
    ex = []
    for _ in range(40):
        st.step(1)
        # uniform up to the cancellation in F(x1) - F(x0) for a 5e-6 cell move
        assert np.ptp(st.E[0]) < 1e-9 * max(1e-30, np.max(np.abs(st.E[0])))
        ex.append(st.E[0].mean())
    ex = np.array(ex)
    ratio = (ex[2:] + ex[:-2]) / ex[1:-1]
    ok = np.abs(ex[1:-1]) > 0.1 * np.max(np.abs(ex))
    assert np.allclose(ratio[ok], 2 - opdt ** 2, rtol=0, atol=1e-8)
    omega = 2 / wl.dt * math.asin(opdt / 2)
    assert omega / wl.omega_pe == pytest.approx(1.0000260, abs=1e-7)


# --------------------------------------------------------------------------
# Q9  vacuum dispersion of the staggered leapfrog (Appendix field solver)
# --------------------------------------------------------------------------

def test_vacuum_dispersion():
    n, dt = 16, 0.45
    g = oracle.Grid(n, n, n, dt)
    kx, ky = 2 * math.pi * 2 / n, 2 * math.pi * 3 / n
    i = np.arange(n)
    # E^z at (i+1/2, j+1/2, k): a transverse standing mode, B = 0
    phase = kx * (i[None, :] + 0.5) + ky * (i[:, None] + 0.5)
    fields = np.zeros((9, n, n, n))
    fields[2] = np.cos(phase)[None, :, :]
    amp = []
    for _ in range(30):
        oracle.half_b(g, fields)
        oracle.half_b(g, fields)
        oracle.update_e(g, fields)
        amp.append(np.sum(fields[2] * np.cos(phase)[None]))
    amp = np.array(amp)
    cos_wdt = 1 - 2 * (dt ** 2) * (math.sin(kx / 2) ** 2 + math.sin(ky / 2) ** 2)
    ratio = (amp[2:] + amp[:-2]) / amp[1:-1]
    ok = np.abs(amp[1:-1]) > 0.1 * np.max(np.abs(amp))
    assert np.allclose(ratio[ok], 2 * cos_wdt, atol=1e-11)


# --------------------------------------------------------------------------
# Q10, Q11  E = -grad_p Phi and B = curl_p A at the particle (Sections 4.2, 4.3)
# --------------------------------------------------------------------------

def _phi_at(g, phi, xp):
    w = oracle.rho_of(g, xp, g.dx * g.dy * g.dz)  # the cell weights dF dF dF
    return np.sum(w * phi)


def test_electric_field_is_gradient_of_potential():
    g = oracle.Grid(6, 5, 7, 0.3, dx=1.1, dy=0.9, dz=1.2)
    phi = RNG.normal(0, 1, g.shape)
    fields = np.zeros((9,) + g.shape)
    fields[0] = (np.roll(phi, 1, axis=2) - phi) / g.dx   # (Phi_{i-1/2} - Phi_{i+1/2})/dx
    fields[1] = (np.roll(phi, 1, axis=1) - phi) / g.dy
    fields[2] = (np.roll(phi, 1, axis=0) - phi) / g.dz
    h = 1e-6
    hs = (g.dx, g.dy, g.dz)
    for _ in range(20):
        xp = RNG.uniform(0, 1, 3) * np.array([6, 5, 7])
        if np.min(np.abs(xp - np.round(xp))) < 1e-3 or np.min(np.abs(xp - np.floor(xp) - 0.5)) < 1e-3:
            continue
        E, _ = oracle.gather(g, fields, xp)
        for a in range(3):
            dp = np.zeros(3)
            dp[a] = h
            grad = (_phi_at(g, phi, xp + dp) - _phi_at(g, phi, xp - dp)) / (2 * h) / hs[a]
            assert E[a] == pytest.approx(-grad, abs=2e-8)


def test_magnetic_field_is_curl_of_vector_potential():
    g = oracle.Grid(6, 7, 5, 0.3, dx=1.0, dy=1.3, dz=0.8)
    A = RNG.normal(0, 1, (3,) + g.shape)
    Ax, Ay, Az = A
    fields = np.zeros((9,) + g.shape)
    fields[3] = (Az - np.roll(Az, 1, axis=1)) / g.dy - (Ay - np.roll(Ay, 1, axis=0)) / g.dz
    fields[4] = (Ax - np.roll(Ax, 1, axis=0)) / g.dz - (Az - np.roll(Az, 1, axis=2)) / g.dx
    fields[5] = (Ay - np.roll(Ay, 1, axis=2)) / g.dx - (Ax - np.roll(Ax, 1, axis=1)) / g.dy
    afields = np.zeros((9,) + g.shape)
    afields[0:3] = A
    hs = (g.dx, g.dy, g.dz)
    h = 1e-6

    def A_at(xp):
        return oracle.gather(g, afields, xp)[0]

    for _ in range(20):
        xp = RNG.uniform(0, 1, 3) * np.array([6, 7, 5])
        if np.min(np.abs(xp - np.round(xp))) < 1e-3 or np.min(np.abs(xp - np.floor(xp) - 0.5)) < 1e-3:
            continue
        _, B = oracle.gather(g, fields, xp)
        d = np.zeros((3, 3))  # d[a][b] = dA_b / dx_a (physical units)
        for a in range(3):
            dp = np.zeros(3)
            dp[a] = h
            d[a] = (A_at(xp + dp) - A_at(xp - dp)) / (2 * h) / hs[a]
        curl = np.array([d[1][2] - d[2][1], d[2][0] - d[0][2], d[0][1] - d[1][0]])
        assert np.allclose(B, curl, atol=2e-8, rtol=0)


# --------------------------------------------------------------------------
# Q12  self-force of a lone 1D sheet (Section 4.4)
# --------------------------------------------------------------------------

def test_self_energy_closed_form():
    se = GOLDEN["self_energy"]
    vals = []
    for d in np.linspace(0, 1, 41):
        xp = 10.0 + d
        nodes = range(6, 16)
        tot = sum((oracle.cumulative1(i - xp) - 0.5) ** 2 / 2 for i in nodes)
        tot -= (len(nodes) - 2) * 0.125  # nodes outside the support contribute (1/2)^2/2 each
        assert tot == pytest.approx(0.125 + 0.25 * d * d * (1 - d) ** 2, abs=1e-15)
        vals.append(tot)
    assert min(vals) == pytest.approx(se["minimum"], abs=1e-15)
    assert max(vals) - min(vals) == pytest.approx(se["variation"], abs=1e-15)


def test_self_force_of_sheet():
    """q sum_i f_i E_i with E_i = 4 pi q dx/V (F_i - 1/2) equals
    -(4 pi q^2 dx / V) d(1-d)(1-2d)/2: zero at d = 0, 1/2 and zero on average."""
    n, q = 32, 0.3
    g = oracle.Grid(n, 1, 1, 0.2, dx=1.0, dy=1.0, dz=1.0)
    forces = []
    ds = np.linspace(0, 1, 201)[:-1]
    for d in ds:
        xp = np.array([16.0 + d, 0.5, 0.5])
        fields = np.zeros((9, 1, 1, n))
        fields[0, 0, 0, :] = [4 * math.pi * q * (oracle.cumulative1(i - xp[0]) - 0.5)
                              for i in range(n)]
        E, _ = oracle.gather(g, fields, xp)
        F = q * E[0]
        assert F == pytest.approx(-4 * math.pi * q * q * 0.5 * d * (1 - d) * (1 - 2 * d),
                                  abs=1e-14)
        forces.append(F)
    assert abs(np.mean(forces)) < 1e-15
    assert abs(forces[0]) < 1e-16 and abs(forces[100]) < 1e-16


def test_lone_particle_with_ion_stays_at_rest():
    g = oracle.Grid(8, 8, 8, 0.45)
    x = np.array([[3.3], [4.6], [2.2]])
    st = oracle.State(g, [oracle.Species(x, np.zeros((3, 1)), np.ones(1)),
                          oracle.Species(x, np.zeros((3, 1)), np.ones(1), q=1.0, mobile=False)])
    st.step(10)
    assert np.all(st.species[0].x == x) and np.all(st.fields == 0.0)


# --------------------------------------------------------------------------
# plane-wave source of the slab workload (total-field / scattered-field)
# --------------------------------------------------------------------------

def test_plane_wave_source_is_one_sided_and_exact():
    """The injected wave exists only in x > plane and there equals the
    auxiliary line's wave at every (y, z): no leakage into the scattered
    region, no transverse structure (until the wave wraps round the box)."""
    n, plane, dt = 128, 8, 0.45   # long box: the precursor must not wrap round
    omega = 2 * math.pi / 20
    g = oracle.Grid(n, 3, 4, dt, source=(plane, omega, omega, 2 * math.pi / omega))
    st = oracle.State(g, [])
    for _ in range(70):   # front travels 0.45 cells/step: no wrap within 70 steps
        st.step(1)
        Ey, Bz = st.fields[1], st.fields[5]
        # round-off leakage only (the grid and line values agree to the last bits)
        assert np.max(np.abs(Ey[:, :, :plane])) < 1e-13 * omega      # faces x = i + 1/2 < plane
        assert np.max(np.abs(Bz[:, :, :plane + 1])) < 1e-13 * omega  # nodes x = i <= plane
        aux_ey = st.aux[:oracle.AUX]
        a = np.arange(plane, n) - (plane - 2)
        assert np.max(np.abs(Ey[:, :, plane:] - aux_ey[a][None, None, :])) < 1e-13 * omega
        for c in (0, 2, 3, 4):
            assert np.max(np.abs(st.fields[c])) == 0.0
    assert np.max(np.abs(st.fields[1])) > 0.5 * omega   # the wave is there (ramp done)


def test_plane_wave_source_amplitude_and_wavelength():
    """The laser as the slab workload's statement fixes it: amplitude a0 = 1,
    i.e. E = a0 omega in units with c = m = |q| = 1, and wavelength 20 cells.
    In vacuum, past the ramp, the injected E^y has amplitude omega, and its
    zeros are half a wavelength apart.  The wavelength is the grid's own,
    from the dispersion relation sin(omega dt / 2) / (c dt) = sin(k dx / 2) / dx
    (19.93 cells for 20 in vacuum).  The phase, a sine from t = 0, is this
    source's convention: the statement does not fix it."""
    n, plane, dt = 256, 8, 0.45
    omega = 2 * math.pi / 20
    ramp = 2 * math.pi / omega
    st = oracle.State(oracle.Grid(n, 2, 2, dt, source=(plane, omega, omega, ramp)), [])
    nsteps = 160
    st.step(nsteps)
    ey = st.fields[1][0, 0, :]
    hi = plane + int((nsteps * dt - ramp) * 0.95)   # launched after the ramp, with a margin
    assert hi - plane > 45
    seg = ey[plane + 2:hi]
    assert np.max(np.abs(seg)) == pytest.approx(omega, rel=0.02)
    k = 2 * np.arcsin(np.sin(omega * dt / 2) / dt)
    i = np.nonzero(np.sign(seg[:-1]) * np.sign(seg[1:]) < 0)[0]
    zeros = i + seg[i] / (seg[i] - seg[i + 1])
    assert len(zeros) >= 4
    assert np.max(np.abs(np.diff(zeros) - np.pi / k)) < 0.05, (np.diff(zeros), np.pi / k)


def test_plane_wave_source_keeps_gauss_and_divb():
    wl = picgen.Workload("src", 24, 6, 6, 3, 0.45, 2, (0.05,) * 3, 0.3, 30)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    omega = 2 * math.pi / 10
    g = oracle.Grid(24, 6, 6, wl.dt, source=(4, omega, omega, 10.0))
    st = oracle.State(g, [oracle.Species(e.x, e.w, e.weight),
                          oracle.Species(ion.x, ion.w, ion.weight, q=1.0, m=100.0, mobile=False)])
    R0 = st.gauss_residual()
    rho_e = np.max(np.abs(4 * np.pi * st.rho(st.species[:1])))
    st.step(30)
    assert np.max(np.abs(st.gauss_residual() - R0)) / rho_e < 1e-12
    assert np.max(np.abs(st.div_b())) < 1e-14
    assert np.max(np.abs(st.fields[1])) > 0.1 * omega


# --------------------------------------------------------------------------
# Electrostatic initial field (Section 4.3, Eqs. poiphi and egradphidis)
# --------------------------------------------------------------------------

def test_poisson_solution_satisfies_gauss_law_and_energy_identity():
    """E = -grad_h Phi of the reference Poisson solve satisfies the discrete
    Gauss law div_h E = 4 pi (rho - <rho>) cell by cell, and the field energy
    equals the potential form printed in Section 4.3:
    V/(8 pi) sum E^2 = (V/2) sum rho Phi."""
    from oracle import poisson
    g = oracle.Grid(10, 7, 6, 0.3, dx=1.1, dy=0.8, dz=1.3)
    rho = RNG.normal(0, 1, g.shape)
    phi = poisson.solve(g, rho)
    E = poisson.e_of_phi(g, phi)
    resid = poisson.div_e(g, E) - 4 * np.pi * (rho - rho.mean())
    assert np.max(np.abs(resid)) < 1e-12 * np.max(np.abs(4 * np.pi * rho))
    V = g.dx * g.dy * g.dz
    lhs = V / (8 * np.pi) * np.sum(E * E)
    rhs = V / 2 * np.sum((rho - rho.mean()) * phi)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_poisson_field_meets_the_step_gauss_law():
    """The reference Poisson field, placed in a particle state, has the step's
    own Gauss residual (Eq. chargelaw, pinned by the whole-run invariants)
    equal to -4 pi <rho> in every cell: the uniform background the solve
    removes.  This ties the module's face convention (E^x between cells i-1
    and i) to the one the step and its deposit use."""
    from oracle import poisson
    wl = picgen.Workload("es", 10, 7, 6, 3, 0.3, 2, (0.1,) * 3, 0.3, 1, seed=12)
    e = picgen.electrons(wl)
    g = oracle.Grid(10, 7, 6, 0.3, dx=1.1, dy=0.8, dz=1.3)
    st = oracle.State(g, [oracle.Species(e.x, e.w, e.weight, q=-1.0, m=1.0)])
    rho = st.rho()
    st.fields[0:3] = poisson.e_of_phi(g, poisson.solve(g, rho))
    R = st.gauss_residual()
    assert np.max(np.abs(R + 4 * np.pi * rho.mean())) < 1e-12 * np.max(np.abs(4 * np.pi * rho))


def test_poisson_single_mode_closed_form():
    """rho = cos(2 pi m x / L) along x: Phi = 4 pi rho / lambda_m with the
    discrete eigenvalue lambda_m = (2 - 2 cos(2 pi m / N)) / dx^2."""
    from oracle import poisson
    n, m, dx = 16, 3, 0.7
    g = oracle.Grid(n, 4, 3, 0.3, dx=dx)
    x = np.arange(n)
    rho = np.broadcast_to(np.cos(2 * np.pi * m * x / n), g.shape).copy()
    phi = poisson.solve(g, rho)
    lam = (2 - 2 * np.cos(2 * np.pi * m / n)) / dx ** 2
    assert np.max(np.abs(phi - 4 * np.pi * rho / lam)) < 1e-12


def test_vector_potential_form_equals_b_form():
    """Advancing A by Eq. dadt and taking B = curl_h A gives the same run as
    advancing B by Eq. updateB (curl_h of the A update is the B update), and
    div_h B stays zero."""
    wl = picgen.Workload("aform", 8, 7, 6, 3, 0.45, 3, (0.2,) * 3, 0.3, 12, seed=9, drift=0.1)
    e = picgen.electrons(wl)
    g = oracle.Grid(8, 7, 6, wl.dt)
    A0 = RNG.normal(0, 1e-3, (3,) + g.shape)
    ref = oracle.State(g, [oracle.Species(e.x, e.w, e.weight, q=-1.0, m=1.0)])
    ref.fields[3:6] = oracle.curl_a(g, A0)
    st = oracle.State(g, [oracle.Species(e.x, e.w, e.weight, q=-1.0, m=1.0)])
    ref.step(wl.steps)
    A = oracle.step_vector_potential(st, A0, wl.steps)
    scale = np.max(np.abs(ref.fields[0:6]))
    assert np.max(np.abs(st.fields[0:6] - ref.fields[0:6])) <= 1e-13 * scale
    assert np.max(np.abs(st.species[0].w - ref.species[0].w)) <= 1e-13
    assert np.max(np.abs(st.div_b())) <= 1e-14 * np.max(np.abs(A)) / 0.5
