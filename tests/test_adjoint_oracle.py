"""Pins of the reference gradient (oracle/adjoint.py), CPU only.

The torch implementation of the step is tied to the C oracle (its forward
state matches after several steps) and its autograd gradient to central
differences of the C oracle's own loss, so the reference gradient of the GPU
adjoint rests on the pinned oracle, not on itself."""
import numpy as np
import pytest

import oracle
import picgen
from oracle import adjoint as ad


def _case(nx, ny, nz, n, seed, w_th=0.1, drift=0.0):
    return picgen.beams((nx, ny, nz), n, seed, w_th=w_th, drift=drift)


def _c_loss(nx, ny, nz, dt, x, w, weight, bext, steps):
    st = oracle.State(oracle.Grid(nx, ny, nz, dt, bext=tuple(bext)),
                      [oracle.Species(x, w, weight, q=-1.0, m=1.0)])
    st.step(steps)
    e = st.energies()
    return e[2] + e[3], st


@pytest.mark.parametrize("dims", [2, 3])
def test_torch_step_matches_c_oracle(dims):
    import torch
    nx, ny, nz = (8, 6, 1) if dims == 2 else (6, 5, 4)
    dt = 0.5 if dims == 2 else 0.45
    x, w, weight = _case(nx, ny, nz, 48, 5 + dims, w_th=0.2)
    if dims == 2:
        x[2] = 0.0
    bext = (0.0, 0.0, 0.05)
    steps = 8
    L, st = _c_loss(nx, ny, nz, dt, x, w, weight, bext, steps)
    g = ad.Grid(nx, ny, nz, dt)
    E = torch.zeros((3, nz, ny, nx), dtype=torch.float64)
    B = torch.zeros_like(E)
    sp = [ad.Species(torch.tensor(x), torch.tensor(w), torch.tensor(weight))]
    E, B, sp = ad.run(g, E, B, sp, torch.tensor(bext, dtype=torch.float64), steps)
    for c in range(3):
        assert np.max(np.abs(E[c].numpy() - st.fields[c])) <= 1e-13 * max(1e-30, np.max(np.abs(st.fields[c])) + 1e-20)
        assert np.max(np.abs(B[c].numpy() - st.fields[3 + c])) <= 1e-13 * (np.max(np.abs(st.fields[3 + c])) + 1e-20)
    d = sp[0].x.numpy() - st.species[0].x
    d -= np.array([nx, ny, nz])[:, None] * np.round(d / np.array([nx, ny, nz])[:, None])
    assert np.max(np.abs(d)) < 1e-12
    assert np.max(np.abs(sp[0].w.numpy() - st.species[0].w)) < 1e-13
    assert abs(float(ad.field_energy(g, E, B)) - L) <= 1e-12 * L


def test_reference_gradient_matches_central_differences_of_c_oracle():
    """dL/dB_ext,z, dL/dw and dL/dx for a few components (2D3V, two
    counter-streaming beams in an external B_z, as the differentiable
    workload) against central differences of the C oracle, h = 1e-6."""
    nx, ny, nz, dt, steps = 8, 8, 1, 0.5, 10
    x, w, weight = _case(nx, ny, nz, 64, 17, w_th=0.05, drift=0.2)
    x[2] = 0.0
    a = 0.05
    L, gw, gb, gx = ad.loss_and_grad(ad.Grid(nx, ny, nz, dt), x, w, weight, -1.0, 1.0, (0.0, 0.0, a), steps)
    L_c, _ = _c_loss(nx, ny, nz, dt, x, w, weight, (0.0, 0.0, a), steps)
    assert abs(L - L_c) <= 1e-12 * L_c
    h = 1e-6
    Lp, _ = _c_loss(nx, ny, nz, dt, x, w, weight, (0.0, 0.0, a + h), steps)
    Lm, _ = _c_loss(nx, ny, nz, dt, x, w, weight, (0.0, 0.0, a - h), steps)
    fd = (Lp - Lm) / (2 * h)
    assert abs(gb[2] - fd) <= 1e-6 * abs(fd) + 1e-9 * L, (gb[2], fd)
    rng = np.random.Generator(np.random.PCG64(3))
    scale = np.max(np.abs(gw))
    for _ in range(4):
        comp, p = int(rng.integers(0, 3)), int(rng.integers(0, x.shape[1]))
        wp, wm = w.copy(), w.copy()
        wp[comp, p] += h
        wm[comp, p] -= h
        fd = (_c_loss(nx, ny, nz, dt, x, wp, weight, (0.0, 0.0, a), steps)[0]
              - _c_loss(nx, ny, nz, dt, x, wm, weight, (0.0, 0.0, a), steps)[0]) / (2 * h)
        assert abs(gw[comp, p] - fd) <= 1e-5 * scale, (comp, p, gw[comp, p], fd)
    scale = np.max(np.abs(gx[:2]))
    for _ in range(4):
        comp, p = int(rng.integers(0, 2)), int(rng.integers(0, x.shape[1]))
        xp, xm = x.copy(), x.copy()
        xp[comp, p] += h
        xm[comp, p] -= h
        fd = (_c_loss(nx, ny, nz, dt, xp, w, weight, (0.0, 0.0, a), steps)[0]
              - _c_loss(nx, ny, nz, dt, xm, w, weight, (0.0, 0.0, a), steps)[0]) / (2 * h)
        assert abs(gx[comp, p] - fd) <= 1e-5 * scale, (comp, p, gx[comp, p], fd)
    assert np.max(np.abs(gx[2])) <= 1e-12 * scale  # z does not enter a 2D step


def _random_fields(shape, seed, amp):
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((9,) + shape)
    f[:6] = rng.normal(0.0, amp, (6,) + shape)
    return f


def test_field_energy_gradient_matches_directional_difference():
    """dL/d(E, B^{n-1/2}) of the field energy against a central difference of
    the C oracle's energy along a random direction."""
    nx, ny, nz, dt = 5, 4, 3, 0.45
    f = _random_fields((nz, ny, nx), 31, 0.3)
    gE, gB = ad.field_energy_grad_fields(ad.Grid(nx, ny, nz, dt), f[:3], f[3:6])
    d = _random_fields((nz, ny, nx), 32, 1.0)
    h = 1e-5

    def energy(ff):
        st = oracle.State(oracle.Grid(nx, ny, nz, dt), [], ff)
        e = st.energies()
        return e[2] + e[3]
    fd = (energy(f + h * d) - energy(f - h * d)) / (2 * h)
    an = np.sum(gE * d[:3]) + np.sum(gB * d[3:6])
    assert abs(an - fd) <= 1e-8 * abs(fd), (an, fd)


@pytest.mark.parametrize("dims", [2, 3])
def test_step_vjp_matches_directional_difference(dims):
    """<lambda', J v> of one step (fields, particles and B_ext perturbed along
    a random direction v) against central differences of the C oracle step."""
    nx, ny, nz = (6, 5, 1) if dims == 2 else (5, 4, 3)
    dt = 0.5 if dims == 2 else 0.45
    n = 40
    x, w, weight = picgen.beams((nx, ny, nz), n, 40 + dims, w_th=0.3, drift=0.2, dims=dims)
    f = _random_fields((nz, ny, nx), 50 + dims, 0.05)
    bext = np.array([0.03, -0.02, 0.05])
    rng = np.random.Generator(np.random.PCG64(60 + dims))
    lam = [rng.normal(size=(3, nz, ny, nx)), rng.normal(size=(3, nz, ny, nx)),
           rng.normal(size=(3, n)), rng.normal(size=(3, n))]
    if dims == 2:
        lam[2][2] = 0.0
    out = ad.step_vjp(ad.Grid(nx, ny, nz, dt), f[:3], f[3:6], x, w, weight, -1.0, 1.0, bext, *lam)
    v = [rng.normal(size=(3, nz, ny, nx)), rng.normal(size=(3, nz, ny, nx)),
         rng.normal(size=(3, n)), rng.normal(size=(3, n)), rng.normal(size=3)]
    if dims == 2:
        v[2][2] = 0.0
    box = np.array([nx, ny, nz], dtype=float)[:, None]

    def functional(s):
        ff = f.copy()
        ff[:3] += s * v[0]
        ff[3:6] += s * v[1]
        st = oracle.State(oracle.Grid(nx, ny, nz, dt, bext=tuple(bext + s * v[4])),
                          [oracle.Species(x + s * v[2], w + s * v[3], weight, q=-1.0, m=1.0)], ff)
        st.step(1)
        # positions enter through their unwrapped displacement from x
        dx = st.species[0].x - x
        dx -= box * np.round(dx / box)
        return (np.sum(lam[0] * st.fields[:3]) + np.sum(lam[1] * st.fields[3:6])
                + np.sum(lam[2] * (x + dx)) + np.sum(lam[3] * st.species[0].w))
    h = 1e-6
    fd = (functional(h) - functional(-h)) / (2 * h)
    an = sum(np.sum(o * d) for o, d in zip(out, v))
    assert abs(an - fd) <= 1e-7 * max(abs(fd), 1.0), (an, fd)


def test_torch_step_with_two_mobile_species_matches_c_oracle():
    """Electrons and mobile positive ions (q = +1, m = 25) in one run: the
    torch restatement equals the C oracle after 8 steps (2D3V)."""
    import torch
    nx, ny, nz, dt, steps = 8, 6, 1, 0.5, 8
    xe, we, wte = _case(nx, ny, nz, 40, 31, w_th=0.2)
    xi, wi, wti = _case(nx, ny, nz, 30, 32, w_th=0.05)
    xe[2] = 0.0
    xi[2] = 0.0
    st = oracle.State(oracle.Grid(nx, ny, nz, dt, bext=(0.0, 0.0, 0.03)),
                      [oracle.Species(xe, we, wte, q=-1.0, m=1.0), oracle.Species(xi, wi, wti, q=1.0, m=25.0)])
    st.step(steps)
    g = ad.Grid(nx, ny, nz, dt)
    E = torch.zeros((3, nz, ny, nx), dtype=torch.float64)
    sp = [ad.Species(torch.tensor(xe), torch.tensor(we), torch.tensor(wte), -1.0, 1.0),
          ad.Species(torch.tensor(xi), torch.tensor(wi), torch.tensor(wti), 1.0, 25.0)]
    E, B, sp = ad.run(g, E, torch.zeros_like(E), sp, torch.tensor([0.0, 0.0, 0.03], dtype=torch.float64), steps)
    assert np.max(np.abs(E.numpy() - st.fields[0:3])) <= 1e-13 * np.max(np.abs(st.fields[0:3]))
    for k in range(2):
        assert np.max(np.abs(sp[k].w.numpy() - st.species[k].w)) < 1e-13
