"""GPU (HIP, gfx950) vs FP64 CPU oracle, element by element, through the C ABI.

Tolerances.  FP64 mode: the GPU evaluates the same formulas in another order
and with fused multiply-adds, so single operations differ in the last bit
(~1e-16 relative); the charge-conserving current differences F(x1) - F(x0)
cancel to the size of one move, amplifying that to ~1e-13 of the current.
Over a run, plasma dynamics amplify differences by a modest factor
(omega_pe t <= 2.5 here).  The bars: relative field error <= 1e-12 (2-norm
over the components of E and of B), particle state <= 1e-12 relative,
Gauss-law drift <= 1e-12 of max |4 pi rho_e|.  FP32 mode is compared with the FP64 oracle and its error
is reported; only the Gauss drift (<= 1e-6) is a hard bar there, plus a loose
bound on the field error stated in each test.
"""
import math

import numpy as np
import pytest

import oracle
import picgen

pytestmark = pytest.mark.gpu


def _sim(**kw):
    from paper_1101_0809_amd import Sim
    return Sim(**kw)


def _rel(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def _wrapdiff(a, b, n):
    d = a - b
    return d - n * np.round(d / n)


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32c", 3e-6)])
@pytest.mark.parametrize("dims", [3, 2])
def test_deposit_matches_oracle(precision, tol, dims):
    """pic_deposit_J of many random moves (several tiles, moves across the
    periodic boundary, a ragged count) equals the oracle's current."""
    n = 16
    nz = n if dims == 3 else 1
    sim = _sim(nx=n, ny=12, nz=nz, dt=0.41, dims=dims, precision=precision,
               dx=1.1, dy=0.9, dz=1.0)
    g = oracle.Grid(n, 12, nz, 0.41, dx=1.1, dy=0.9, dz=1.0)
    x0, x1 = picgen.random_moves(1237, seed=5, box=(n, 12, nz), max_step=0.9)
    if dims == 2:
        x1[2] = x0[2] + (x1[2] - x0[2]) * 0.5
    if precision == "fp32c":
        # the FP32 path represents positions as cell + FP32 offset: give both
        # sides the same representable start and displacement
        x0 = np.floor(x0) + (x0 - np.floor(x0)).astype(np.float32).astype(np.float64)
        x1 = x0 + (x1 - x0).astype(np.float32).astype(np.float64)
    q = np.random.Generator(np.random.PCG64(6)).uniform(-1, 1, x0.shape[1])
    J = sim.deposit(x0, x1, q).cpu().numpy()
    ref = np.zeros((3,) + g.shape)
    for p in range(x0.shape[1]):
        oracle.deposit(g, x0[:, p], x1[:, p], q[p], J=ref)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(J - ref)) / scale < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32c", 3e-6)])
@pytest.mark.parametrize("dims", [3, 2])
def test_deposit_degenerate_moves(precision, tol, dims):
    """pic_deposit_J on the method's degenerate moves: starts and ends exactly
    on cell faces (offset 0), moves onto a face from either side, no move,
    single-axis moves, a move ending exactly on the periodic boundary and
    one leaving cell 0 downwards.  Integer and half-integer positions are
    exact in FP32 too, so both precisions take the same inputs."""
    n, ny = 16, 12
    nz = n if dims == 3 else 1
    box = np.array([n, ny, nz], dtype=float)[:, None]
    rng = np.random.Generator(np.random.PCG64(7))
    m = 64
    cells = np.stack([rng.integers(0, b, m) for b in (n, ny, nz)]).astype(float)
    half = rng.integers(-1, 2, (3, m)) * 0.5            # -0.5, 0, 0.5 per axis
    frac = np.round(rng.uniform(0.05, 0.95, (3, m)) * 64) / 64
    moves = []
    moves.append((cells, cells + half))                  # face to face or to a mid-point
    moves.append((cells + frac, np.floor(cells + frac)))  # onto the face below
    moves.append((cells + frac, np.ceil(cells + frac)))   # onto the face above
    moves.append((cells + frac, cells + frac))            # no move
    for a in range(3):                                    # one axis at a time
        x1 = cells + frac
        x1 = x1.copy()
        x1[a] = np.floor(x1[a]) if a % 2 else np.ceil(x1[a])
        moves.append((cells + frac, x1))
    edge0 = cells + frac
    edge0[0] = n - 0.25
    edge1 = edge0.copy()
    edge1[0] = float(n)                                   # exactly onto the periodic boundary
    moves.append((edge0, edge1))
    low0 = cells + frac
    low0[0] = 0.0
    low1 = low0.copy()
    low1[0] = -0.375                                      # from cell 0's lower face downwards
    moves.append((low0, low1))
    x0 = np.concatenate([a for a, _ in moves], axis=1)
    x1 = np.concatenate([b for _, b in moves], axis=1)
    if dims == 2:   # as in the random-move test: the z displacement halved
        x1[2] = x0[2] + (x1[2] - x0[2]) * 0.5
    assert np.all(np.abs(x1 - x0) < 1.0)
    sim = _sim(nx=n, ny=ny, nz=nz, dt=0.41, dims=dims, precision=precision)
    g = oracle.Grid(n, ny, nz, 0.41)
    q = rng.uniform(-1, 1, x0.shape[1])
    J = sim.deposit(x0, x1, q).cpu().numpy()
    ref = np.zeros((3,) + g.shape)
    for p in range(x0.shape[1]):
        oracle.deposit(g, x0[:, p], x1[:, p], q[p], J=ref)
    scale = np.max(np.abs(ref))
    assert scale > 0
    assert np.max(np.abs(J - ref)) / scale < tol
    # a particle that does not move carries no current
    still = np.zeros(x0.shape[1], bool)
    k = 3 * m
    still[k:k + m] = True
    Js = sim.deposit(x0[:, still], x1[:, still], q[still]).cpu().numpy()
    assert np.max(np.abs(Js)) == 0.0


def test_field_solve_matches_oracle():
    n = (10, 9, 8)
    rng = np.random.Generator(np.random.PCG64(3))
    fields = rng.normal(0, 1, (9, n[2], n[1], n[0]))
    sim = _sim(nx=n[0], ny=n[1], nz=n[2], dt=0.45, dims=3, dx=1.0, dy=1.2, dz=0.9, fields=fields)
    g = oracle.Grid(*n, 0.45, dx=1.0, dy=1.2, dz=0.9)
    ref = fields.copy()
    sim.field_solve("b_half")
    oracle.half_b(g, ref)
    assert np.max(np.abs(sim.fields_numpy() - ref)) < 1e-14
    sim.field_solve("e_full")
    oracle.half_b(g, ref)
    oracle.update_e(g, ref)
    ref[6:9] = 0.0
    assert np.max(np.abs(sim.fields_numpy() - ref)) < 1e-13


# ---------------------------------------------------------------------------
# whole runs
# ---------------------------------------------------------------------------

def _run_pair(wl, precision, steps, sort_every=None, ions=True):
    e = picgen.electrons(wl)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision=precision,
               sort_every=wl.sort_every if sort_every is None else sort_every, bext=wl.bext)
    se = sim.add_species(e.q, e.m, e.n)
    sim.load(se, e.x, e.w, e.weight)
    species = [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m)]
    if ions:
        ion = picgen.ions_like(wl, e)
        si = sim.add_species(ion.q, ion.m, 0, mobile=False)
        sim.load(si, ion.x, ion.w, ion.weight)
        species.append(oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False))
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext), species)
    sim.step(steps)
    st.step(steps)
    return sim, st, e


def _compare(sim, st, wl, field_tol, part_tol, gauss_tol):
    """Field error per vector field, ||F_gpu - F_ref|| / ||F_ref|| over the three
    components of E and of B, <= field_tol; a single small component (a
    longitudinal field beside a strong laser) is allowed 100x that, since
    its error is set by the rounding of the large components' currents."""
    F = sim.fields_numpy()
    for name, sl in (("E", slice(0, 3)), ("B", slice(3, 6))):
        err = _rel(F[sl], st.fields[sl])
        assert err <= field_tol, (name, err)
    for c, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz"]):
        err = _rel(F[c], st.fields[c])
        assert err <= 100 * field_tol, (name, err)
    x, w, _, ids = sim.particles(0)
    sp = st.species[0]
    dims = wl.dims
    for a, n in enumerate((wl.nx, wl.ny, wl.nz)[:dims]):
        dx = _wrapdiff(x[a], sp.x[a], n)
        assert np.max(np.abs(dx)) <= part_tol * n, ("x", a, np.max(np.abs(dx)))
    werr = np.max(np.abs(w - sp.w)) / np.max(np.abs(sp.w))
    assert werr <= part_tol, ("w", werr)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= gauss_tol, d
    assert d["nonfinite"] == 0
    # the oracle's own Gauss drift, for reference
    return d


def test_2d3v_32x32_fp64_parity():
    """The 32x32 2D3V parity workload: 4096 electrons, 100 steps, FP64."""
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"]
    sim, st, _ = _run_pair(wl, "fp64", wl.steps, sort_every=10)
    _compare(sim, st, wl, 1e-12, 1e-12, 1e-12)


def test_3d_small_fp64_parity():
    """3D, 16^3 cells (8 tiles) x 8 per cell, 20 steps, re-sorted every 5 steps
    (so particles drift out of their tiles between sorts)."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=16, ny=16, nz=16, steps=20, sort_every=5)
    sim, st, _ = _run_pair(wl, "fp64", wl.steps)
    _compare(sim, st, wl, 1e-12, 1e-12, 1e-12)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_ragged_tiles_parity(precision, tols):
    """Cell counts that are not multiples of the tile (partial tiles), hot
    plasma so many particles take the out-of-tile path, no re-sort.  The grid
    is narrower than a tile's LDS regions (in FP32 mode the x field region
    spans 14 cells of a 13-cell axis), so staging and flush wrap onto the
    same cells."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=13, ny=10, nz=11, w_th=(0.5, 0.5, 0.5),
                                                  ppc=3, steps=12, sort_every=0)
    sim, st, _ = _run_pair(wl, precision, wl.steps)
    assert sim.fallback_fraction() > 0.0 or sim.migrant_fraction() > 0.0
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_migrants_and_full_buckets_parity(precision, tols):
    """A beam at w_x = 1 (0.32 cells per step) that is sorted only when loaded:
    after 18 steps a large share of the electrons is beyond their sorted
    tile's region (the immobile ions left behind pull the beam back; the
    oracle's trajectories put 38% of the next 4 steps' updates there in FP32
    mode, whose region is widest) and is advanced by the migrant pass of the
    tile it moved into.  The species' capacity equals its
    count, so each of the 16 tiles' buckets holds a quarter of the particles,
    and the two tiles the beam (y < 8) enters overflow: their extra migrants
    take the global-memory path.  Against the oracle."""
    rng = np.random.Generator(np.random.PCG64(4242))
    nx, ny, nz = 32, 16, 16
    n = 4 * 4 * 8 * nz
    x = np.stack([4.0 + 4.0 * rng.random(n), 8.0 * rng.random(n), nz * rng.random(n)])
    w = rng.normal(0.0, 0.05, (3, n))
    w[0] += 1.0
    weight = np.full(n, 0.002)
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=0.45, dims=3, precision=precision, sort_every=0)
    se = sim.add_species(-1.0, 1.0, n)
    sim.load(se, x, w, weight)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, x, np.zeros_like(w), weight)
    st = oracle.State(oracle.Grid(nx, ny, nz, 0.45),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0),
                       oracle.Species(x, np.zeros_like(w), weight, q=1.0, m=100.0, mobile=False)])
    sim.step(18)
    st.step(18)
    sim.step(4)   # statistics of the last call: much of the beam is beyond its tiles' regions
    st.step(4)
    mig, fb = sim.migrant_fraction(), sim.fallback_fraction()
    assert mig > 0.3 and fb > 0.0, (mig, fb)
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=nx, ny=ny, nz=nz)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_tile_margin_along_x(precision, tols):
    """The tile region's margin along x: 3 cells in FP32 mode, 1 in FP64.  A
    light beam (its own field negligible) starts in the last x cell of its
    tile (x in [7.15, 7.25)) at w_x = 1 (0.318 cells per step; a transverse
    spread of 0.01 makes every field component physical) and is sorted
    only when loaded.  Steps 7 and 8 start with every particle in cell 9, two
    cells past its tile: inside the FP32 region, so no particle is a migrant;
    outside the FP64 one, so every particle is (the capacity leaves room in
    the one bucket they all enter).  Steps 11 and 12 start in cell 10, the
    FP32 region's last; steps 14 and 15 in cell 11, past it, where every
    particle is a migrant in both modes.  Against the oracle."""
    rng = np.random.Generator(np.random.PCG64(4343))
    nx, ny, nz, n = 32, 16, 16, 2000
    x = np.stack([7.15 + 0.1 * rng.random(n), 8.0 * rng.random(n), 8.0 * rng.random(n)])
    w = rng.normal(0.0, 0.01, (3, n))
    w[0] += 1.0
    weight = np.full(n, 1e-6)
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=0.45, dims=3, precision=precision, sort_every=0)
    se = sim.add_species(-1.0, 1.0, 16 * n)
    sim.load(se, x, w, weight)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, x, np.zeros_like(w), weight)
    st = oracle.State(oracle.Grid(nx, ny, nz, 0.45),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0),
                       oracle.Species(x, np.zeros_like(w), weight, q=1.0, m=100.0, mobile=False)])
    sim.step(6)
    st.step(6)
    xs = sim.particles(0)[0]
    assert np.all((xs[0] >= 9.0) & (xs[0] < 9.25)), (xs[0].min(), xs[0].max())
    sim.step(2)   # statistics of this call: the steps that start in cell 9
    st.step(2)
    mig = sim.migrant_fraction()
    if precision == "fp32c":
        assert mig == 0.0, mig
    else:
        assert mig > 0.99, mig
    sim.step(2)   # steps 9 and 10: the beam enters cell 10
    st.step(2)
    assert np.all(np.floor(sim.particles(0)[0][0]) == 10.0)
    sim.step(2)   # steps 11 and 12 start in cell 10
    st.step(2)
    mig = sim.migrant_fraction()
    if precision == "fp32c":
        assert mig == 0.0, mig
    else:
        assert mig > 0.99, mig
    sim.step(1)   # step 13: the beam enters cell 11
    st.step(1)
    assert np.all(np.floor(sim.particles(0)[0][0]) == 11.0)
    sim.step(2)   # steps 14 and 15 start in cell 11, past every region
    st.step(2)
    assert sim.migrant_fraction() > 0.99
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=nx, ny=ny, nz=nz)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_face_and_centre_starts(precision, tols):
    """Particles that start exactly on cell faces (integer coordinates, offset
    0: node factors (1, 0), cell factors (1/2, 1/2, 0)) or at cell centres
    (offset 1/2), half of them at rest, among a random third; the immobile
    ions sit at the electrons' starts.  10 steps, re-sorted every 4, against
    the oracle."""
    rng = np.random.Generator(np.random.PCG64(4646))
    nx, ny, nz, m = 16, 16, 16, 3000
    cells = np.stack([rng.integers(0, b, m) for b in (nx, ny, nz)]).astype(float)
    x = np.concatenate([cells[:, :1000], cells[:, 1000:2000] + 0.5,
                        cells[:, 2000:] + rng.random((3, 1000))], axis=1)
    w = rng.normal(0.0, 0.2, (3, m))
    w[:, ::2] = 0.0   # every other particle at rest
    weight = np.full(m, 0.01)
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=0.45, dims=3, precision=precision, sort_every=4)
    se = sim.add_species(-1.0, 1.0, m)
    sim.load(se, x, w, weight)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, x, np.zeros_like(w), weight)
    st = oracle.State(oracle.Grid(nx, ny, nz, 0.45),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0),
                       oracle.Species(x, np.zeros_like(w), weight, q=1.0, m=100.0, mobile=False)])
    sim.step(10)
    st.step(10)
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=nx, ny=ny, nz=nz)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("axis,dims3", [(0, (2048, 16, 16)), (1, (16, 2048, 16)), (2, (16, 16, 1024))])
@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_largest_axis_wrap(precision, tols, axis, dims3):
    """The largest axes the FP32 cell word holds (11 + 11 + 10 bits: 2048
    cells along x and y, 1024 along z).  A light beam starts in the last two
    cells of the long axis at 1 c (0.32 cells per step) and crosses its
    periodic boundary, so the highest packed cell index and its wrap to
    cell 0 are stored, sorted (every 3 steps) and advanced.  Against the
    oracle."""
    rng = np.random.Generator(np.random.PCG64(4545 + axis))
    n = 2000
    L = dims3[axis]
    x = np.stack([dims3[a] * rng.random(n) for a in range(3)])
    x[axis] = (L - 1.6) + 1.5 * rng.random(n)
    w = rng.normal(0.0, 0.01, (3, n))
    w[axis] += 1.0
    weight = np.full(n, 1e-4)
    nx, ny, nz = dims3
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=0.45, dims=3, precision=precision, sort_every=3)
    se = sim.add_species(-1.0, 1.0, n)
    sim.load(se, x, w, weight)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, x, np.zeros_like(w), weight)
    st = oracle.State(oracle.Grid(nx, ny, nz, 0.45),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0),
                       oracle.Species(x, np.zeros_like(w), weight, q=1.0, m=100.0, mobile=False)])
    sim.step(9)
    st.step(9)
    xs = sim.particles(0)[0][axis]
    assert np.mean(xs < 3.0) > 0.95, np.mean(xs < 3.0)   # the beam wrapped to the start of the axis
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=nx, ny=ny, nz=nz)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_3d_crowded_cell_parity(precision, tols):
    """600 electrons packed in one cell, beamed along +x, among a uniform
    background: a wave chunk holds far more particles of one lane class
    than its 16 class rows, so the rest run in the unordered tail, and the
    crowd's crossers share one window class, so their column of the crossing
    map overflows and the entries outside it deposit in arrival order --
    against the oracle, with re-sorts inside the run."""
    rng = np.random.Generator(np.random.PCG64(20260))
    n = 16
    crowd = 600
    x = np.concatenate([5.0 + rng.random((3, crowd)), rng.random((3, 1000)) * n], axis=1)
    beam = rng.normal(0.0, 0.05, (3, crowd))
    beam[0] += 0.9  # crossers of the crowd share one window class
    w = np.concatenate([beam, rng.normal(0.0, 0.1, (3, 1000))], axis=1)
    weight = np.full(x.shape[1], 0.01)
    sim = _sim(nx=n, ny=n, nz=n, dt=0.45, dims=3, precision=precision, sort_every=3)
    se = sim.add_species(-1.0, 1.0, x.shape[1])
    sim.load(se, x, w, weight)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, x, np.zeros_like(w), weight)
    st = oracle.State(oracle.Grid(n, n, n, 0.45),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0),
                       oracle.Species(x, np.zeros_like(w), weight, q=1.0, m=100.0, mobile=False)])
    sim.step(7)
    st.step(7)
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=n, ny=n, nz=n)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("dims", [2, 3])
def test_fp32c_against_fp64_oracle(dims):
    """FP32 mode vs the FP64 oracle: Gauss drift <= 1e-6 (hard), field and
    particle errors within the FP32 rounding envelope (reported)."""
    if dims == 2:
        wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(steps=40)
    else:
        wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=16, ny=16, nz=16, steps=20, sort_every=5)
    sim, st, _ = _run_pair(wl, "fp32c", wl.steps)
    d = _compare(sim, st, wl, 1e-3, 1e-5, 1e-6)
    print("fp32c", dims, d)


def test_2d_kernel_equals_3d_kernel_with_one_z_cell():
    """The 2D3V kernels equal the 3D kernels run on an nz = 1 grid (every z sum
    of a partition of unity is one)."""
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(steps=10)
    e = picgen.electrons(wl)
    out = []
    for dims in (2, 3):
        sim = _sim(nx=wl.nx, ny=wl.ny, nz=1, dt=wl.dt, dims=dims, sort_every=5)
        s = sim.add_species(e.q, e.m, e.n)
        sim.load(s, e.x, e.w, e.weight)
        sim.step(wl.steps)
        x, w, _, _ = sim.particles(0)
        out.append((sim.fields_numpy(), x, w))
    (F2, x2, w2), (F3, x3, w3) = out
    for c in range(6):
        assert _rel(F2[c], F3[c]) < 1e-14 or np.max(np.abs(F3[c])) == 0
    assert np.max(np.abs(_wrapdiff(x2[:2], x3[:2], 32))) < 1e-13
    assert np.max(np.abs(w2 - w3)) < 1e-14 * np.max(np.abs(w3))


def test_gyration_on_gpu():
    """A lone electron in a uniform external B with the gyration parameters of
    Section 5 (omega_B dt = 0.25, |w| = 0.5 c, c dt/dx = 0.5) moves on the
    closed-form circle through the full GPU step; its weight is 1e-30 so its
    own current leaves the fields at round-off level."""
    dt = 0.025
    dx = 2 * dt
    n = 32
    sim = _sim(nx=n, ny=n, nz=n, dt=dt, dims=3, dx=dx, dy=dx, dz=dx, bext=(0.0, 0.0, 10.0))
    s = sim.add_species(-1.0, 1.0, 1)
    sim.load(s, np.array([[16.0], [16.0], [16.0]]), np.array([[0.5], [0.0], [0.0]]),
             np.array([1e-30]))
    pts = []
    for _ in range(64):
        sim.step(1)
        pts.append(sim.particles(0)[0][:, 0])
    pts = np.array(pts)
    gam = math.sqrt(1.25)
    theta = 2 * math.atan(0.25 / (2 * gam))
    R = (0.5 / gam) * dt / (2 * math.sin(theta / 2)) / dx
    a, b, c = pts[0, :2], pts[1, :2], pts[2, :2]
    d = 2 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
    ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
    uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
    r = np.hypot(pts[:, 0] - ux, pts[:, 1] - uy)
    assert np.max(np.abs(r - R)) < 1e-11
    # Eq. (1): dw/dt = (q/m)(u/c x B); with q < 0 and B along +z the electron
    # turns counter-clockwise seen from +z, theta per step
    ang = np.unwrap(np.arctan2(pts[:, 1] - uy, pts[:, 0] - ux))
    assert np.allclose(np.diff(ang), theta, atol=1e-11)


def test_load_rejects_out_of_range():
    from paper_1101_0809_amd import PicError
    sim = _sim(nx=8, ny=8, nz=8, dt=0.4, dims=3)
    s = sim.add_species(-1.0, 1.0, 4)
    x = np.array([[1.0, 2.0, 8.0, 3.0], [1.0, 1.0, 1.0, 1.0], [1.0, 1.0, 1.0, 1.0]])
    with pytest.raises(PicError) as ei:
        sim.load(s, x, np.zeros((3, 4)), np.ones(4))
    assert ei.value.code == -2
    assert sim.count(s) == 0


def test_empty_species_and_zero_steps():
    sim = _sim(nx=8, ny=8, nz=8, dt=0.4, dims=3)
    sim.add_species(-1.0, 1.0, 16)
    sim.step(0)
    sim.step(3)
    d = sim.diagnostics()
    assert d["n_particles"] == 0 and d["gauss_abs"] == 0.0
    assert np.all(sim.fields_numpy() == 0.0)


# ---------------------------------------------------------------------------
# the full-size 64^3 x 8 workload (the benchmark configuration), sampled
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_64cube_fullsize_sampled(precision):
    """Full 64^3 x 8 per cell (2,097,152 electrons) in the launch
    configuration the benchmark times: after 20 steps (two re-sorts), one more
    step is checked particle by particle on a sample against the oracle's
    single-particle step using the GPU's own pre-step fields; the Gauss drift
    holds over the whole grid."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"]
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=64, ny=64, nz=64, dt=wl.dt, dims=3, precision=precision, sort_every=10)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    sim.step(20)
    fields = sim.fields_numpy()
    x0, w0, wt, ids = sim.particles(0)
    sim.step(1)
    x1, w1, _, ids1 = sim.particles(0)
    assert np.array_equal(ids, ids1)
    g = oracle.Grid(64, 64, 64, wl.dt)
    bn = fields.copy()
    oracle.half_b(g, bn)
    rng = np.random.Generator(np.random.PCG64(99))
    sample = rng.choice(e.n, 3000, replace=False)
    tol = 1e-12 if precision == "fp64" else 2e-6
    for p in sample:
        E, B = oracle.gather(g, bn, x0[:, p])
        wn = oracle.push(-1.0, wl.dt, 1.0, E, B, w0[:, p])
        xn = x0[:, p] + oracle.displacement(g, wn)
        assert np.max(np.abs(wn - w1[:, p])) <= tol * max(1e-3, np.max(np.abs(wn)))
        assert np.max(np.abs(_wrapdiff(xn, x1[:, p], 64))) <= tol * 64
    d = sim.diagnostics()
    assert d["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6), d
    assert d["nonfinite"] == 0
    assert abs(d["charge"]) < 1e-9 * e.n * e.weight[0]


@pytest.mark.parametrize("dims,precision", [(3, "fp64"), (3, "fp32c"), (2, "fp64")])
def test_sort_order(dims, precision):
    """After a sort, storage order is tile-major and the ids are a permutation
    of the loaded ones.  Inside a 3D tile of n_t particles, slot s holds a
    particle of lane class s mod C (C = 16 FP64, 32 FP32; the class of tile
    cell l is its field-tile base index mod C: ((lx+2) + 14 (ly+2) + 168 (lz+2))
    in FP64, ((lx+4) + 18 (ly+2) + 216 (lz+2)) in FP32) in as many slots as the
    class counts allow -- sum over classes of min(count, rows of the column) --
    those slots form the first rows of each column, and down a column the
    cells follow their (lz, ly) row order.  Inside a 2D tile: rank levels in
    order, cells in row-major order within a level."""
    if dims == 3:
        wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=20, ny=16, nz=9, steps=0)
        T = 8
    else:
        wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(nx=40, ny=20, ppc=6)
        T = 16
    e = picgen.electrons(wl)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=dims, precision=precision)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    sim.sort()
    x, _, _, ids = sim.particles(0, raw=True)
    assert np.array_equal(np.sort(ids), np.arange(e.n))
    cell = np.floor(x).astype(np.int64)
    nt = [(wl.nx + T - 1) // T, (wl.ny + T - 1) // T, (wl.nz + T - 1) // T if dims == 3 else 1]
    tz = cell[2] // T if dims == 3 else np.zeros_like(cell[0])
    tile = (tz * nt[1] + cell[1] // T) * nt[0] + cell[0] // T
    assert np.all(np.diff(tile) >= 0)
    lz = cell[2] % T if dims == 3 else np.zeros_like(cell[0])
    lx, ly = cell[0] % T, cell[1] % T
    if dims == 3:
        if precision == "fp64":
            C, cls = 16, ((lx + 2) + 14 * (ly + 2) + 168 * (lz + 2)) % 16
        else:
            C, cls = 32, ((lx + 4) + 18 * (ly + 2) + 216 * (lz + 2)) % 32
        row_order = lz * T + ly
        for t in np.unique(tile):
            sel = np.flatnonzero(tile == t)
            n_t = sel.size
            k = cls[sel]
            slot = np.arange(n_t)
            counts = np.bincount(k, minlength=C)
            rows = np.array([max(0, -(-(n_t - c) // C)) for c in range(C)])
            home = k == slot % C
            assert home.sum() == np.minimum(counts, rows).sum()
            for c in range(C):
                col = slot % C == c
                h = home[col]
                m = int(min(counts[c], rows[c]))
                assert h[:m].all() and not h[m:].any()
                ro = row_order[sel][col][:m]
                assert np.all(np.diff(ro) >= 0)
    else:
        local = ly * T + lx
        for t in np.unique(tile):
            loc = local[tile == t]
            # a new rank level starts exactly where the local cell index drops
            level = np.concatenate([[0], np.cumsum(np.diff(loc) <= 0)])
            for lv in np.unique(level):
                cells = loc[level == lv]
                assert np.all(np.diff(cells) > 0)
            # level r holds one particle of every cell with more than r particles
            counts = np.bincount(loc, minlength=T ** dims)
            for lv in np.unique(level):
                assert np.sum(level == lv) == np.sum(counts > lv)


def _sampled_step_check(sim, g, qm, dims, n_axis, tol, rng_seed=99, nsample=2000, species=0):
    """Read the state, take one GPU step, and compare a sample of particles with
    the oracle's single-particle step from the GPU's own pre-step fields."""
    import torch
    fields = sim.fields_numpy()
    n = sim.count(species)
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    sample = np.sort(rng.choice(n, nsample, replace=False))   # particle ids

    def read():
        """Sampled particles by id (the storage order may change at a sort)."""
        import ctypes
        x = torch.empty((3, n), dtype=torch.float64, device=sim.device)
        w = torch.empty((3, n), dtype=torch.float64, device=sim.device)
        pid = torch.empty(n, dtype=torch.int64, device=sim.device)
        sim._check(sim.lib.pic_get_particles(sim.ctx, species, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(w.data_ptr()), None,
                                              ctypes.c_void_p(pid.data_ptr()),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        where = torch.empty(n, dtype=torch.int64, device=sim.device)
        where[pid] = torch.arange(n, device=sim.device)
        idx = where[torch.as_tensor(sample, device=sim.device)]
        out = (x[:, idx].cpu().numpy(), w[:, idx].cpu().numpy(), pid[idx].cpu().numpy())
        del x, w, pid, where
        return out

    x0, w0, id0 = read()
    sim.step(1)
    x1, w1, id1 = read()
    assert np.array_equal(id0, sample) and np.array_equal(id1, sample)
    bn = fields.copy()
    oracle.half_b(g, bn)
    for k in range(nsample):
        E, B = oracle.gather(g, bn, x0[:, k])
        wn = oracle.push(qm, g.dt, 1.0, E, B, w0[:, k])
        xn = x0[:, k] + oracle.displacement(g, wn)
        assert np.max(np.abs(wn - w1[:, k])) <= tol * max(1e-3, np.max(np.abs(wn))), k
        for a in range(dims):
            assert abs(_wrapdiff(xn[a], x1[a, k], n_axis[a])) <= tol * n_axis[a], (k, a)


_FULL64 = {}


def _oracle_64cube_12_steps(wl):
    """The oracle's 12 steps of the full 64^3 x 8 workload, run once and
    shared by both precisions (about 30 s of CPU)."""
    if "st" not in _FULL64:
        e = picgen.electrons(wl)
        ion = picgen.ions_like(wl, e)
        st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, bext=wl.bext),
                          [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m),
                           oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False)])
        st.step(wl.steps)
        _FULL64["st"] = st
    return _FULL64["st"]


@pytest.mark.parametrize("precision,tols", [("fp64", (1e-12, 1e-12, 1e-12)),
                                             ("fp32c", (1e-3, 1e-5, 1e-6))])
def test_64cube_fullsize_elementwise(precision, tols):
    """The 64^3 x 8 workload (2,097,152 electrons, co-located ions) at full
    size: 12 steps across the sort at step 10, then all six field planes and
    every particle (by id) against the oracle's 12 steps, in FP64 and in FP32
    mode (against the same FP64 oracle run)."""
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(steps=12)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=wl.dims, precision=precision,
               sort_every=wl.sort_every, bext=wl.bext)
    se = sim.add_species(e.q, e.m, e.n)
    sim.load(se, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    sim.step(wl.steps)
    st = _oracle_64cube_12_steps(wl)
    _compare(sim, st, wl, *tols)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_256sq_beams_fullsize_sampled(precision):
    """The 256^2 2D3V two-stream workload (1,048,576 electrons, drifts +-0.2 c,
    external B_z = omega_pe) at full size: 40 steps (two re-sorts), then a
    sampled single-step check against the oracle and the Gauss drift."""
    wl = picgen.WORKLOADS["2d3v_256sq_beams"]
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=1, dt=wl.dt, dims=2, precision=precision,
               sort_every=wl.sort_every, bext=wl.bext)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    sim.step(39)
    g = oracle.Grid(wl.nx, wl.ny, 1, wl.dt, bext=wl.bext)
    _sampled_step_check(sim, g, -1.0, 2, (wl.nx, wl.ny, 1),
                        1e-12 if precision == "fp64" else 2e-6)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6), d
    assert d["nonfinite"] == 0


@pytest.mark.parametrize("precision,tol,gauss_tol", [("fp32c", 2e-6, 1e-6), ("fp64", 1e-12, 1e-12)])
def test_256cube_weibel_fullsize_sampled(precision, tol, gauss_tol):
    """The 256^3 anisotropic workload at full size, in FP32 mode (the headline)
    and in FP64 (155 GB of particle buffers): 536,870,912 electrons (w_th =
    0.3, 0.05, 0.05) and as many mobile ions (M = 100), drawn on the GPU.  A
    sampled single-step check of both species against the oracle, and the
    Gauss drift."""
    import torch
    wl = picgen.WORKLOADS["3d_256cube_weibel"]
    dev = torch.device("cuda:0")
    sim = _sim(nx=256, ny=256, nz=256, dt=wl.dt, dims=3, precision=precision,
               sort_every=wl.sort_every)
    n = wl.n_electrons
    se = sim.add_species(-1.0, 1.0, n)
    si = sim.add_species(1.0, wl.ion_mass, n)
    for sp, ions in ((se, False), (si, True)):
        for x, w, wt in picgen.device_chunks(wl, dev, ions=ions):
            sim.load(sp, x, w, wt)
            del x, w, wt
    torch.cuda.empty_cache()
    assert sim.count(se) == n and sim.count(si) == n
    sim.step(2)
    g = oracle.Grid(256, 256, 256, wl.dt)
    # sampled checks, electrons then ions (one more step is taken inside each)
    _sampled_step_check(sim, g, -1.0, 3, (256, 256, 256), tol, nsample=800, species=se)
    _sampled_step_check(sim, g, 1.0 / wl.ion_mass, 3, (256, 256, 256), tol, nsample=800, species=si)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= gauss_tol, d
    assert d["nonfinite"] == 0 and d["n_particles"] == 2 * n


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_checkpoint_restore_continue(precision, tmp_path):
    """Save after 12 steps (mid sort period), restore into a fresh context and
    continue 8 steps: same result as running 20 steps straight, up to the
    summation order of the atomics."""
    import torch
    from paper_1101_0809_amd import Sim
    wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=16, ny=16, nz=16, sort_every=5)
    e = picgen.electrons(wl)
    sim = _sim(nx=16, ny=16, nz=16, dt=wl.dt, dims=3, precision=precision, sort_every=5)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    sim.step(12)
    path = tmp_path / "ckpt.pt"
    torch.save(sim.state_dict(), path)
    sim.step(8)
    ref_f = sim.fields_numpy()
    ref_x, ref_w, _, _ = sim.particles(0)
    sim2 = Sim.from_state_dict(torch.load(path, weights_only=True))
    sim2.step(8)
    f = sim2.fields_numpy()
    x, w, _, _ = sim2.particles(0)
    assert sim2.diagnostics()["step"] == 20
    tol = 1e-12 if precision == "fp64" else 1e-5
    for c in range(6):
        assert _rel(f[c], ref_f[c]) < tol
    assert np.max(np.abs(w - ref_w)) < tol * np.max(np.abs(ref_w))
    assert np.max(np.abs(_wrapdiff(x, ref_x, 16))) < tol * 16


# ---------------------------------------------------------------------------
# plane-wave source (the laser of the 128^3 slab workload)
# ---------------------------------------------------------------------------

def _slab_oracle_state(wl, source, e=None):
    e = picgen.electrons(wl) if e is None else e
    ion = picgen.ions_like(wl, e)
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, source=source),
                      [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m),
                       oracle.Species(ion.x, ion.w, ion.weight, q=ion.q, m=ion.m, mobile=False)])
    return st, e, ion


def test_plane_wave_source_vacuum_matches_oracle():
    omega = 2 * math.pi / 20
    src = (8, omega, omega, 20.0)
    sim = _sim(nx=64, ny=8, nz=8, dt=0.45, dims=3, source=src)
    st = oracle.State(oracle.Grid(64, 8, 8, 0.45, source=src), [])
    sim.step(60)
    st.step(60)
    F = sim.fields_numpy()
    for c in range(6):
        assert np.max(np.abs(F[c] - st.fields[c])) <= 1e-13 * omega, c
    aux = sim.aux_line()
    assert np.max(np.abs(aux - st.aux)) <= 1e-13 * omega
    assert np.max(np.abs(F[1])) > 0.5 * omega


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_slab_with_laser_parity(precision):
    """The slab workload at reduced size (48 x 16 x 16 cells, electrons at 8 per
    cell in x in [12, 36), cold, immobile ions) with the laser plane at x = 4:
    40 steps against the oracle, in a periodic box (the open x form is in
    test_gpu_open_x.py)."""
    wl = picgen.WORKLOADS["3d_128cube_slab"].scaled(nx=48, ny=16, nz=16, ppc=8, slab=(12, 36),
                                                   steps=40, sort_every=10)
    omega = 2 * math.pi / 20
    src = (4, omega, omega, 20.0)
    st, e, ion = _slab_oracle_state(wl, src)
    sim = _sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=3, precision=precision,
               sort_every=wl.sort_every, source=src)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    sim.step(wl.steps)
    st.step(wl.steps)
    if precision == "fp64":
        _compare(sim, st, wl, 1e-12, 1e-12, 1e-12)
    else:
        _compare(sim, st, wl, 1e-4, 1e-5, 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_128cube_slab_laser_fullsize_sampled(precision):
    """The full 128^3 slab workload: 16 electrons per slab cell in x in [32, 96)
    (16,777,216 electrons), w_th = 0.01 c, a0 = 1 laser of 20-cell wavelength
    from the plane x = 8 with a one-period sin^2 ramp.  After 60 steps the
    wave has entered the plasma; one more step is checked on a sample against
    the oracle, and the Gauss drift over the grid.  The box is periodic here;
    the workload's own open x walls are in test_gpu_open_x.py."""
    wl = picgen.WORKLOADS["3d_128cube_slab"]
    omega = 2 * math.pi / 20
    src = (8, omega, omega, 20.0)
    e = picgen.electrons(wl)
    ion = picgen.ions_like(wl, e)
    sim = _sim(nx=128, ny=128, nz=128, dt=wl.dt, dims=3, precision=precision,
               sort_every=wl.sort_every, source=src)
    s = sim.add_species(e.q, e.m, e.n)
    sim.load(s, e.x, e.w, e.weight)
    si = sim.add_species(ion.q, ion.m, 0, mobile=False)
    sim.load(si, ion.x, ion.w, ion.weight)
    del e, ion
    sim.step(59)
    g = oracle.Grid(128, 128, 128, wl.dt)   # the source only acts on the grid
    _sampled_step_check(sim, g, -1.0, 3, (128, 128, 128),
                        1e-12 if precision == "fp64" else 2e-6, nsample=1500)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6), d
    assert d["nonfinite"] == 0
    assert d["field_e"] > 0.0


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_residual_diagnostics_match_oracle(precision):
    """pic_diagnostics' charge and field checks against the oracle's own
    definitions -- the Gauss residual R = div_h E - 4 pi rho (Eq. chargelaw)
    with rho of Eq. rho, div_h B at the nodes, the total charge -- on a state
    where every one of them is far from zero: random initial E and B (so R^0
    and div B are non-zero), hot electrons and an immobile background placed
    apart from them (net charge), a ragged grid of several tiles.  After the
    steps E is overwritten in the GPU's field buffer with a perturbed copy,
    so that R^n - R^0 is non-zero as well.  The oracle evaluates everything
    from the GPU's fields and stored particles; both sides are FP64."""
    import torch
    rng = np.random.Generator(np.random.PCG64(777))
    nx, ny, nz, dt = 13, 10, 11, 0.45
    F0 = np.zeros((9, nz, ny, nx))
    F0[:6] = rng.normal(0.0, 1e-3, (6, nz, ny, nx))
    ne, ni = 3000, 2000
    xe = np.stack([rng.uniform(0, nn, ne) for nn in (nx, ny, nz)])
    we = rng.normal(0.0, 0.3, (3, ne))
    wte = np.full(ne, 0.01)
    xi = np.stack([rng.uniform(0, nn, ni) for nn in (nx, ny, nz)])
    wti = np.full(ni, 0.013)
    sim = _sim(nx=nx, ny=ny, nz=nz, dt=dt, dims=3, precision=precision, sort_every=4, fields=F0)
    se = sim.add_species(-1.0, 1.0, ne)
    sim.load(se, xe, we, wte)
    si = sim.add_species(1.0, 100.0, 0, mobile=False)
    sim.load(si, xi, np.zeros_like(xi), wti)
    x0, _, w0, _ = sim.particles(se)            # the stored start state (FP32 mode: rounded)
    sim.step(6)
    F = sim.fields_numpy()
    F[0:3] += rng.normal(0.0, 1e-4, (3, nz, ny, nx))
    sim.fields[0:3].copy_(torch.from_numpy(np.ascontiguousarray(F[0:3])).to(sim.device))
    d = sim.diagnostics()
    x1, _, w1, _ = sim.particles(se)
    g = oracle.Grid(nx, ny, nz, dt)
    wti_stored = wti.astype(np.float32).astype(np.float64) if precision == "fp32c" else wti
    ions = oracle.Species(xi, np.zeros_like(xi), wti_stored, q=1.0, m=100.0, mobile=False)
    rho_bg = oracle.State(g, [ions]).rho()
    rho_m0 = oracle.State(g, [oracle.Species(x0, np.zeros_like(x0), w0, q=-1.0)]).rho()
    rho_m1 = oracle.State(g, [oracle.Species(x1, np.zeros_like(x1), w1, q=-1.0)]).rho()
    R0 = oracle.State(g, [], fields=F0).gauss_residual(rho_m0 + rho_bg)
    st1 = oracle.State(g, [], fields=F)
    R1 = st1.gauss_residual(rho_m1 + rho_bg)
    gauss_abs = np.max(np.abs(R1 - R0))
    rho_max = np.max(np.abs(4 * np.pi * rho_m1))
    divb = np.max(np.abs(st1.div_b()))
    charge = np.sum(rho_m1 + rho_bg)
    assert gauss_abs > 1e-4 and divb > 1e-4 and abs(charge) > 1.0   # all far from zero
    assert d["gauss_abs"] == pytest.approx(gauss_abs, rel=1e-12)
    assert d["rho_mobile_max"] == pytest.approx(rho_max, rel=1e-12)
    assert d["gauss_rel"] == pytest.approx(gauss_abs / rho_max, rel=1e-12)
    assert d["divb_max"] == pytest.approx(divb, rel=1e-12)
    assert d["charge"] == pytest.approx(charge, rel=1e-12)
    assert d["nonfinite"] == 0 and d["n_particles"] == ne


@pytest.mark.parametrize("dims", [3, 2])
@pytest.mark.parametrize("scheme", ["alternating-1", "alternating-2", "conventional"])
def test_energy_diagnostics_match_oracle(scheme, dims):
    """pic_diagnostics' energies (kinetic at t^{n-1/2}, the half-step term
    (q dt / 2) u . E(x^n) with the run's own gather, E and B^n field energies,
    Section 4.1) against the oracle's, after a run with fields grown from a
    drifting plasma."""
    order = 2 if scheme == "alternating-2" else 1
    interp = "conventional" if scheme == "conventional" else "alternating"
    if dims == 3:
        wl = picgen.WORKLOADS["3d_64cube_8ppc"].scaled(nx=12, ny=10, nz=9, ppc=3, steps=15, sort_every=5,
                                                      drift=0.1)
    else:
        wl = picgen.WORKLOADS["2d3v_32x32_fp64"].scaled(nx=24, ny=20, steps=30, sort_every=5, drift=0.1)
    e = picgen.electrons(wl)
    from paper_1101_0809_amd import Sim
    sim = Sim(nx=wl.nx, ny=wl.ny, nz=wl.nz, dt=wl.dt, dims=dims, sort_every=wl.sort_every, order=order,
              interp=interp)
    sim.add_species(e.q, e.m, e.n)
    sim.load(0, e.x, e.w, e.weight)
    st = oracle.State(oracle.Grid(wl.nx, wl.ny, wl.nz, wl.dt, order=order, interp=1 if interp == "conventional" else 0),
                      [oracle.Species(e.x, e.w, e.weight, q=e.q, m=e.m)])
    sim.step(wl.steps)
    st.step(wl.steps)
    d = sim.diagnostics()
    ref = st.energies()
    assert abs(d["kinetic"] - ref[0]) <= 1e-12 * ref[0]
    assert abs(d["kinetic_half_step"] - ref[1]) <= 1e-10 * abs(ref[1]) + 1e-14 * ref[0], (d["kinetic_half_step"], ref[1])
    assert abs(d["field_e"] - ref[2]) <= 1e-11 * ref[2]
    assert abs(d["field_b"] - ref[3]) <= 1e-11 * ref[3] + 1e-14 * ref[2]
    sim.close()
