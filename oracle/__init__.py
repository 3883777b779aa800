"""Double-precision CPU oracle of the charge-conserving PIC step (arXiv:1101.0809).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It wraps the
plain C reference in ``pic_oracle.c`` with ctypes (argument marshalling only)
and shares no code with the GPU library.

Arrays follow the C conventions: fields are ``(9, nz, ny, nx)`` float64 in
the order Ex Ey Ez Bx By Bz Jx Jy Jz; positions and momenta are ``(3, n)``
float64 (cell units, momentum over mass); weights ``(n,)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


AUX = 8192  # auxiliary line length of the plane-wave source (ORC_AUX)
ABSORB = 2  # particle-absorbing layer at each open x wall, in cells (ORC_ABSORB)


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("bext", ctypes.c_double * 3),
                ("src_kind", ctypes.c_int64), ("src_plane", ctypes.c_int64),
                ("src_amp", ctypes.c_double), ("src_omega", ctypes.c_double),
                ("src_ramp", ctypes.c_double), ("order", ctypes.c_int64),
                ("interp", ctypes.c_int64), ("xbc", ctypes.c_int64)]


class _Species(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("mobile", ctypes.c_int32), ("deposit", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("w", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.c_double
        p = ctypes.c_void_p
        g = ctypes.POINTER(_Grid)
        s = ctypes.POINTER(_Species)
        sig = {
            "orc_shape": (d, [ctypes.c_int, d]),
            "orc_cumulative1": (d, [d]),
            "orc_cumulative2": (d, [d]),
            "orc_gather": (None, [g, p, p, p, p]),
            "orc_push": (None, [d, d, d, p, p, p]),
            "orc_displacement": (None, [g, p, p]),
            "orc_deposit": (None, [g, p, p, d, p]),
            "orc_deposit_quarter": (None, [g, p, p, d, p]),
            "orc_rho_add": (None, [g, p, d, p]),
            "orc_rho": (None, [g, ctypes.c_int, s, p]),
            "orc_half_b": (None, [g, p]),
            "orc_update_e": (None, [g, p]),
            "orc_particle_step": (None, [g, p, s, p]),
            "orc_step": (None, [g, p, ctypes.c_int, s, ctypes.c_int]),
            "orc_step_src": (None, [g, p, ctypes.c_int, s, ctypes.c_int, p, ctypes.c_int64]),
            "orc_gauss_residual": (None, [g, p, p, p]),
            "orc_div_b": (None, [g, p, p]),
            "orc_energies": (None, [g, p, ctypes.c_int, s, p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous and a.dtype == np.float64
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dt: float
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    c: float = 1.0
    bext: tuple = (0.0, 0.0, 0.0)
    source: tuple = None   # (plane, amplitude, omega, ramp time): +x plane wave, E^y
    order: int = 1         # alternating order l_a = order + 1/2 (Section 4.5): 1 or 2
    interp: int = 0        # 0 alternating order; 1 the conventional uniform order (Eq. wrong1)
    xbc: int = 0           # x boundary: 0 periodic; 1 open (Mur walls at x = 0 and nx - 1,
                           # particles absorbed within ABSORB cells of a wall)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    def _c(self) -> _Grid:
        g = _Grid()
        g.nx, g.ny, g.nz = self.nx, self.ny, self.nz
        g.dx, g.dy, g.dz, g.dt, g.c = self.dx, self.dy, self.dz, self.dt, self.c
        g.order = int(self.order)
        g.interp = int(self.interp)
        g.xbc = int(self.xbc)
        for a in range(3):
            g.bext[a] = float(self.bext[a])
        if self.source is not None:
            g.src_kind = 1
            g.src_plane, g.src_amp, g.src_omega, g.src_ramp = (int(self.source[0]),
                                                               *map(float, self.source[1:]))
        return g


@dataclass
class Species:
    x: np.ndarray          # (3, n) positions, cell units
    w: np.ndarray          # (3, n) momentum over mass at n-1/2
    weight: np.ndarray     # (n,)
    q: float = -1.0        # charge per unit weight
    m: float = 1.0         # mass per unit weight
    mobile: bool = True
    deposit: bool = True

    def __post_init__(self):
        self.x = _f64(self.x).reshape(3, -1).copy()
        self.w = _f64(self.w).reshape(3, -1).copy()
        self.weight = _f64(self.weight).reshape(-1).copy()
        assert self.x.shape[1] == self.w.shape[1] == self.weight.shape[0]

    @property
    def n(self):
        return self.weight.shape[0]

    def _c(self) -> _Species:
        s = _Species()
        s.n, s.q, s.m = self.n, self.q, self.m
        s.mobile, s.deposit = int(self.mobile), int(self.deposit)
        s.x, s.w, s.weight = _ptr(self.x), _ptr(self.w), _ptr(self.weight)
        return s


def _species_array(species):
    arr = (_Species * max(1, len(species)))()
    for i, s in enumerate(species):
        arr[i] = s._c()
    return arr


@dataclass
class State:
    """E^n, B^{n-1/2} (and J^{n-1/2}) on the grid plus the particle species."""
    grid: Grid
    species: list = field(default_factory=list)
    fields: np.ndarray = None

    step_index: int = 0

    def __post_init__(self):
        if self.fields is None:
            self.fields = np.zeros((9,) + self.grid.shape)
        self.fields = _f64(self.fields).copy()
        self.aux = np.zeros(2 * AUX)   # source line: E^y then B^z

    @property
    def E(self):
        return self.fields[0:3]

    @property
    def B(self):
        return self.fields[3:6]

    @property
    def J(self):
        return self.fields[6:9]

    def step(self, nsteps: int = 1):
        lib().orc_step_src(ctypes.byref(self.grid._c()), _ptr(self.fields),
                           len(self.species), _species_array(self.species), nsteps,
                           _ptr(self.aux), self.step_index)
        self.step_index += nsteps

    def rho(self, species=None):
        sp = self.species if species is None else species
        out = np.zeros(self.grid.shape)
        lib().orc_rho(ctypes.byref(self.grid._c()), len(sp), _species_array(sp), _ptr(out))
        return out

    def gauss_residual(self, rho=None):
        rho = self.rho() if rho is None else _f64(rho)
        out = np.zeros(self.grid.shape)
        lib().orc_gauss_residual(ctypes.byref(self.grid._c()), _ptr(self.fields), _ptr(rho),
                                 _ptr(out))
        return out

    def div_b(self):
        out = np.zeros(self.grid.shape)
        lib().orc_div_b(ctypes.byref(self.grid._c()), _ptr(self.fields), _ptr(out))
        return out

    def energies(self):
        """(kinetic, half-step term, electric, magnetic at B^n)."""
        out = np.zeros(4)
        lib().orc_energies(ctypes.byref(self.grid._c()), _ptr(self.fields),
                           len(self.species), _species_array(self.species), _ptr(out))
        return out


# --- single-particle entry points (used by the pins) ------------------------

def shape(l: int, r: float) -> float:
    return lib().orc_shape(l, r)


def cumulative1(s: float) -> float:
    return lib().orc_cumulative1(s)


def cumulative2(s: float) -> float:
    return lib().orc_cumulative2(s)


def gather(grid: Grid, fields: np.ndarray, xp):
    fields = _f64(fields)
    xp = _f64(xp).copy()
    E = np.zeros(3)
    B = np.zeros(3)
    lib().orc_gather(ctypes.byref(grid._c()), _ptr(fields), _ptr(xp), _ptr(E), _ptr(B))
    return E, B


def push(q_over_m: float, dt: float, c: float, Ep, Bp, w):
    w = _f64(w).copy()
    Ep, Bp = _f64(Ep).copy(), _f64(Bp).copy()  # keep the buffers alive across the call
    lib().orc_push(q_over_m, dt, c, _ptr(Ep), _ptr(Bp), _ptr(w))
    return w


def displacement(grid: Grid, w):
    out = np.zeros(3)
    w = _f64(w).copy()
    lib().orc_displacement(ctypes.byref(grid._c()), _ptr(w), _ptr(out))
    return out


def deposit(grid: Grid, x0, x1, charge: float, J=None, form: str = "sixth"):
    J = np.zeros((3,) + grid.shape) if J is None else J
    fn = lib().orc_deposit if form == "sixth" else lib().orc_deposit_quarter
    x0, x1 = _f64(x0).copy(), _f64(x1).copy()
    fn(ctypes.byref(grid._c()), _ptr(x0), _ptr(x1), charge, _ptr(J))
    return J


def rho_of(grid: Grid, xp, charge: float):
    out = np.zeros(grid.shape)
    xp = _f64(xp).copy()
    lib().orc_rho_add(ctypes.byref(grid._c()), _ptr(xp), charge, _ptr(out))
    return out


def half_b(grid: Grid, fields: np.ndarray):
    lib().orc_half_b(ctypes.byref(grid._c()), _ptr(fields))


def update_e(grid: Grid, fields: np.ndarray):
    lib().orc_update_e(ctypes.byref(grid._c()), _ptr(fields))


# --- vector-potential form (Section 4.2, Eq. dadt) ---------------------------

def curl_a(grid: Grid, A: np.ndarray) -> np.ndarray:
    """B (3, nz, ny, nx) = curl_h A on the staggered grid: B^x at (i+1/2, j, k)
    from A^z at j -+ 1/2 and A^y at k -+ 1/2, and cyclic (A stored like E)."""
    Ax, Ay, Az = A
    r = lambda a, ax: np.roll(a, 1, axis=ax)  # value at index - 1 along ax
    return np.stack([(Az - r(Az, 1)) / grid.dy - (Ay - r(Ay, 0)) / grid.dz,
                     (Ax - r(Ax, 0)) / grid.dz - (Az - r(Az, 2)) / grid.dx,
                     (Ay - r(Ay, 2)) / grid.dx - (Ax - r(Ax, 1)) / grid.dy])


def step_vector_potential(st: "State", A: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance a state in the vector-potential form: before each step B^{n-1/2}
    is curl_h A^{n-1/2}; after it A^{n+1/2} = A^{n-1/2} - c dt E^n with the
    E^n the step started from.  Returns A after the steps; the state's B is
    curl_h of it."""
    A = np.array(A, dtype=np.float64)
    for _ in range(nsteps):
        st.fields[3:6] = curl_a(st.grid, A)
        E = st.fields[0:3].copy()
        st.step(1)
        A = A - st.grid.c * st.grid.dt * E
    st.fields[3:6] = curl_a(st.grid, A)
    return A
