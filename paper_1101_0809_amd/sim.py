"""Thin Python front end of the gfx950 PIC library.

PyTorch provides the device memory (every buffer is a torch tensor on the
GPU) and the stream (torch's current stream); each method marshals pointers
and sizes into one C-ABI call of ``include/pic.h``.  No step of the method
runs in Python.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _align(n: int, a: int = 256) -> int:
    return (n + a - 1) // a * a


def _dev_f64(a, device) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64))
    return t.to(device=device, dtype=torch.float64).contiguous()


@dataclass
class SpeciesInfo:
    index: int
    q: float
    m: float
    mobile: bool
    capacity: int
    buffer: torch.Tensor = None


class Sim:
    """One simulation context: grid, fields and particle species on one GPU.

    Positions are in cell units, momenta are w = gamma v (momentum over
    mass); see include/pic.h for the conventions.
    """

    def __init__(self, nx: int, ny: int, nz: int, dt: float, dims: int = 3,
                 precision: str = "fp64", dx: float = 1.0, dy: float = 1.0, dz: float = 1.0,
                 c: float = 1.0, sort_every: int = 0, bext=(0.0, 0.0, 0.0),
                 device: str = "cuda:0", fields: np.ndarray = None, source=None, order: int = 1,
                 interp: str = "alternating", field_form: str = "B", xbc: str = "periodic"):
        """source: None or (plane, amplitude, omega, ramp time) for the +x
        E^y plane-wave source of include/pic.h.  order: alternating form
        factor order l_a = order + 1/2 (1, or 2 in FP64).  interp:
        "alternating" or "conventional" (the uniform-order comparison of
        Eq. wrong1; order 1, FP64).  field_form: "B", or "A" to carry the
        vector potential (Section 4.2, Eq. dadt) with B = curl_h A.  xbc:
        "periodic", or "open" for Mur walls at x = 0 and x = nx - 1 and
        particles absorbed within PIC_ABSORB cells of them (include/pic.h)."""
        if not torch.cuda.is_available():
            raise RuntimeError("the PIC library needs a GPU (no CPU fallback)")
        self.lib = L.load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        d = L.GridDesc()
        d.dims, d.nx, d.ny, d.nz = dims, nx, ny, nz
        d.precision = {"fp64": L.PIC_FP64, "fp32c": L.PIC_FP32C}[precision]
        d.order, d.sort_every = int(order), sort_every
        d.interp = {"alternating": 0, "conventional": 1}[interp]
        d.field_form = {"B": 0, "A": 1}[field_form]
        d.xbc = {"periodic": 0, "open": 1}[xbc]
        d.dx, d.dy, d.dz, d.dt, d.c = dx, dy, dz, dt, c
        for a in range(3):
            d.bext[a] = float(bext[a])
        if source is not None:
            d.src_kind, d.src_plane = 1, int(source[0])
            d.src_amp, d.src_omega, d.src_ramp = (float(v) for v in source[1:])
        self.desc = d
        self.precision = precision
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        sz = L.Sizes()
        L.check(self.lib.pic_query_sizes(ctypes.byref(d), 0, ctypes.byref(sz)))
        self.fields_t = torch.zeros(9 * self.ncell, dtype=torch.float64, device=self.device)
        if fields is not None:
            self.fields_t.copy_(_dev_f64(fields, self.device).reshape(-1))
        self.workspace = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        torch.cuda.synchronize()
        L.check(self.lib.pic_init_grid(ctypes.byref(d), ctypes.c_void_p(self.fields_t.data_ptr()),
                                       sz.field_bytes, ctypes.c_void_p(self.workspace.data_ptr()),
                                       sz.workspace_bytes, ctypes.byref(ctx)))
        self.ctx = ctx
        self.species = []

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            torch.cuda.synchronize()
            self.lib.pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        L.check(rc, self.ctx)

    # -- particles -------------------------------------------------------
    def add_species(self, q: float, m: float, capacity: int, mobile: bool = True) -> int:
        s = L.SpeciesDesc()
        s.q, s.m, s.mobile, s.reserved, s.capacity = q, m, int(mobile), 0, capacity
        buf = None
        nbytes = 0
        if mobile:
            sz = L.Sizes()
            L.check(self.lib.pic_query_sizes(ctypes.byref(self.desc), capacity, ctypes.byref(sz)))
            buf = torch.empty(sz.particle_bytes, dtype=torch.uint8, device=self.device)
            nbytes = sz.particle_bytes
        idx = ctypes.c_int()
        self._check(self.lib.pic_add_species(
            self.ctx, ctypes.byref(s), ctypes.c_void_p(buf.data_ptr() if buf is not None else 0),
            nbytes, ctypes.byref(idx)))
        self.species.append(SpeciesInfo(idx.value, q, m, mobile, capacity, buf))
        return idx.value

    def load(self, species: int, x, w, weight):
        """Append particles: x, w of shape (3, n) (cell units, momentum over
        mass), weight (n,).  Host (numpy) or device arrays."""
        x = x if isinstance(x, torch.Tensor) else _dev_f64(x, self.device)
        w = w if isinstance(w, torch.Tensor) else _dev_f64(w, self.device)
        weight = weight if isinstance(weight, torch.Tensor) else _dev_f64(weight, self.device)
        x, w, weight = (t.to(self.device, torch.float64).contiguous() for t in (x, w, weight))
        n = weight.numel()
        assert x.numel() == 3 * n and w.numel() == 3 * n
        self._check(self.lib.pic_load_particles(
            self.ctx, species, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
            ctypes.c_void_p(weight.data_ptr()), _stream()))

    def count(self, species: int = 0) -> int:
        return int(self.lib.pic_particle_count(self.ctx, species))

    def particles(self, species: int = 0, raw: bool = False):
        """Return (x, w, weight, id) as host numpy arrays in id order (in the
        library's storage order when raw is true)."""
        n = self.count(species)
        x = torch.empty((3, n), dtype=torch.float64, device=self.device)
        w = torch.empty((3, n), dtype=torch.float64, device=self.device)
        wt = torch.empty(n, dtype=torch.float64, device=self.device)
        pid = torch.empty(n, dtype=torch.int64, device=self.device)
        self._check(self.lib.pic_get_particles(
            self.ctx, species, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
            ctypes.c_void_p(wt.data_ptr()), ctypes.c_void_p(pid.data_ptr()), _stream()))
        torch.cuda.synchronize()
        if raw:
            return x.cpu().numpy(), w.cpu().numpy(), wt.cpu().numpy(), pid.cpu().numpy()
        order = torch.argsort(pid)
        return (x[:, order].cpu().numpy(), w[:, order].cpu().numpy(),
                wt[order].cpu().numpy(), pid[order].cpu().numpy())

    # -- stepping --------------------------------------------------------
    def step(self, nsteps: int = 1):
        self._check(self.lib.pic_step(self.ctx, nsteps, _stream()))

    def sort(self):
        self._check(self.lib.pic_sort(self.ctx, _stream()))

    def field_solve(self, what: str):
        op = {"b_half": L.PIC_B_HALF, "e_full": L.PIC_E_FULL}[what]
        self._check(self.lib.pic_field_solve(self.ctx, op, _stream()))

    def deposit(self, x0, x1, charge) -> torch.Tensor:
        """Current J (3, nz, ny, nx) of particles moving x0 -> x1 (arrays (3, n))."""
        x0 = _dev_f64(x0, self.device) if not isinstance(x0, torch.Tensor) else x0.contiguous()
        x1 = _dev_f64(x1, self.device) if not isinstance(x1, torch.Tensor) else x1.contiguous()
        q = _dev_f64(charge, self.device) if not isinstance(charge, torch.Tensor) else charge.contiguous()
        J = torch.zeros((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.pic_deposit_J(
            self.ctx, ctypes.c_void_p(x0.data_ptr()), ctypes.c_void_p(x1.data_ptr()),
            ctypes.c_void_p(q.data_ptr()), q.numel(), ctypes.c_void_p(J.data_ptr()), _stream()))
        return J

    def solve_poisson(self, neutralize: bool = True, tol: float = 1e-13):
        """E from the discrete Poisson equation of the current charge
        (include/pic.h, pic_solve_poisson); returns (iterations, relative
        residual)."""
        it = ctypes.c_int64()
        res = ctypes.c_double()
        self._check(self.lib.pic_solve_poisson(self.ctx, int(neutralize), tol, ctypes.byref(it),
                                               ctypes.byref(res), _stream()))
        return it.value, res.value

    def set_vector_potential(self, A):
        """A^{n-1/2} (3, nz, ny, nx) of a field_form "A" context; B becomes curl_h A."""
        A = A if isinstance(A, torch.Tensor) else _dev_f64(A, self.device)
        A = A.to(self.device, torch.float64).contiguous()
        assert A.numel() == 3 * self.ncell
        self._check(self.lib.pic_set_vector_potential(self.ctx, ctypes.c_void_p(A.data_ptr()), _stream()))
        torch.cuda.current_stream().synchronize()

    def vector_potential(self) -> np.ndarray:
        A = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.pic_get_vector_potential(self.ctx, ctypes.c_void_p(A.data_ptr()), _stream()))
        torch.cuda.synchronize()
        return A.cpu().numpy()

    def diagnostics(self) -> dict:
        d = L.Diag()
        self._check(self.lib.pic_diagnostics(self.ctx, ctypes.byref(d), _stream()))
        return d.as_dict()

    def diagnostics_static(self) -> dict:
        """pic_diagnostics_static: the same diagnostics with the library's
        static scratch instead of the context's workspace."""
        d = L.Diag()
        self._check(self.lib.pic_diagnostics_static(self.ctx, ctypes.byref(d), _stream()))
        return d.as_dict()

    def timing_start(self, max_steps: int):
        self._check(self.lib.pic_timing_start(self.ctx, max_steps))

    def timing_stop(self):
        """Summed event times (ms) of the recorded steps: dict with b_half,
        particles, e_update, sort and the number of steps."""
        ms = (ctypes.c_double * 4)()
        n = ctypes.c_int64()
        self._check(self.lib.pic_timing_stop(self.ctx, ms, ctypes.byref(n)))
        return {"b_half": ms[0], "particles": ms[1], "e_update": ms[2], "sort": ms[3],
                "steps": n.value}

    def fallback_fraction(self) -> float:
        return float(self.lib.pic_last_fallback_fraction(self.ctx, _stream()))

    def migrant_fraction(self) -> float:
        return float(self.lib.pic_last_migrant_fraction(self.ctx, _stream()))

    # -- checkpoint ------------------------------------------------------
    def state_dict(self) -> dict:
        """Everything needed to continue the run: byte copies of the caller
        buffers (fields, workspace, particle buffers) and the host state."""
        hs = L.HostState()
        self._check(self.lib.pic_get_host_state(self.ctx, ctypes.byref(hs)))
        torch.cuda.synchronize()
        return {
            "desc": {name: (list(getattr(self.desc, name)) if name == "bext"
                            else getattr(self.desc, name)) for name, _ in L.GridDesc._fields_},
            "fields": self.fields_t.clone(),
            "workspace": self.workspace.clone(),
            "species": [{"q": s.q, "m": s.m, "mobile": s.mobile, "capacity": s.capacity,
                         "buffer": None if s.buffer is None else s.buffer.clone()}
                        for s in self.species],
            "host": {"step": hs.step, "since_sort": hs.since_sort, "r0_valid": hs.r0_valid,
                     "nsp": hs.nsp, "n": list(hs.n), "sorted": list(hs.sorted),
                     "copy": list(hs.copy)},
        }

    @classmethod
    def from_state_dict(cls, st: dict, device: str = "cuda:0") -> "Sim":
        d = st["desc"]
        prec = {L.PIC_FP64: "fp64", L.PIC_FP32C: "fp32c"}[d["precision"]]
        src = ((d["src_plane"], d["src_amp"], d["src_omega"], d["src_ramp"])
               if d["src_kind"] == 1 else None)
        sim = cls(d["nx"], d["ny"], d["nz"], d["dt"], dims=d["dims"], precision=prec,
                  dx=d["dx"], dy=d["dy"], dz=d["dz"], c=d["c"], sort_every=d["sort_every"],
                  bext=tuple(d["bext"]), device=device, source=src, order=d["order"],
                  interp=("alternating", "conventional")[d["interp"]],
                  field_form=("B", "A")[d["field_form"]],
                  xbc=("periodic", "open")[d.get("xbc", 0)])
        for sp in st["species"]:
            sim.add_species(sp["q"], sp["m"], sp["capacity"], mobile=sp["mobile"])
        sim.fields_t.copy_(st["fields"])
        sim.workspace.copy_(st["workspace"])
        for mine, sp in zip(sim.species, st["species"]):
            if sp["buffer"] is not None:
                mine.buffer.copy_(sp["buffer"])
        h = st["host"]
        hs = L.HostState()
        hs.step, hs.since_sort, hs.r0_valid, hs.nsp = h["step"], h["since_sort"], h["r0_valid"], h["nsp"]
        for i in range(4):
            hs.n[i], hs.sorted[i], hs.copy[i] = h["n"][i], h["sorted"][i], h["copy"][i]
        torch.cuda.synchronize()
        sim._check(sim.lib.pic_set_host_state(sim.ctx, ctypes.byref(hs)))
        return sim

    # -- adjoint ---------------------------------------------------------
    def snapshot(self) -> dict:
        """Device copies of the caller buffers and the host state, for
        restore() on this same context (no host round trip)."""
        hs = L.HostState()
        self._check(self.lib.pic_get_host_state(self.ctx, ctypes.byref(hs)))
        return {"fields": self.fields_t.clone(), "workspace": self.workspace.clone(),
                "buffers": [None if s.buffer is None else s.buffer.clone() for s in self.species],
                "host": hs}

    def restore(self, snap: dict):
        """Put the context back into the state snapshot() recorded."""
        self.fields_t.copy_(snap["fields"])
        self.workspace.copy_(snap["workspace"])
        for s, b in zip(self.species, snap["buffers"]):
            if b is not None:
                s.buffer.copy_(b)
        hs = L.HostState.from_buffer_copy(snap["host"])
        self._check(self.lib.pic_set_host_state(self.ctx, ctypes.byref(hs)))

    def adjoint_seed_field_energy(self, lam_fields: torch.Tensor):
        """Write d(field energy)/d(E^n, B^{n-1/2}) into lam_fields (6 N FP64)."""
        assert lam_fields.dtype == torch.float64 and lam_fields.numel() == 6 * self.ncell
        self._check(self.lib.pic_adjoint_seed_field_energy(
            self.ctx, ctypes.c_void_p(lam_fields.data_ptr()), _stream()))

    def adjoint_record_bytes(self) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.pic_adjoint_record_bytes(self.ctx, ctypes.byref(n)))
        return n.value

    def adjoint_record(self, record: torch.Tensor):
        """Copy the state the next step starts from into record (a uint8
        device tensor of adjoint_record_bytes())."""
        self._check(self.lib.pic_adjoint_record(self.ctx, ctypes.c_void_p(record.data_ptr()),
                                                record.numel(), _stream()))

    def _lam_ptrs(self, lam_x, lam_w):
        nsp = len(self.species)
        px = (ctypes.c_void_p * nsp)()
        pw = (ctypes.c_void_p * nsp)()
        for i, s in enumerate(self.species):
            if s.mobile:
                n = self.count(i)
                for t in (lam_x[i], lam_w[i]):
                    assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == 3 * n
                px[i], pw[i] = lam_x[i].data_ptr(), lam_w[i].data_ptr()
        return px, pw

    def host_state(self):
        hs = L.HostState()
        self._check(self.lib.pic_get_host_state(self.ctx, ctypes.byref(hs)))
        return hs

    def set_host_state(self, hs):
        self._check(self.lib.pic_set_host_state(self.ctx, ctypes.byref(hs)))

    def adjoint_reorder(self, src, dst, lam_x: list, lam_w: list, out_x: list, out_w: list):
        """Particle adjoints from the storage order of record src to that of
        record dst (None: id order), out of place."""
        px, pw = self._lam_ptrs(lam_x, lam_w)
        ox, ow = self._lam_ptrs(out_x, out_w)
        nb = src.numel() if src is not None else (dst.numel() if dst is not None else 0)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
        self._check(self.lib.pic_adjoint_reorder(self.ctx, ptr(src), ptr(dst), nb, px, pw, ox, ow, _stream()))

    def adjoint_step_record(self, record: torch.Tensor, lam_fields: torch.Tensor, lam_x: list,
                            lam_w: list, lam_bext: torch.Tensor, ordered: bool = False):
        """adjoint_step with the state before the step taken from a record;
        ordered: particle adjoints by position in the record instead of id."""
        px, pw = self._lam_ptrs(lam_x, lam_w)
        assert lam_fields.numel() == 6 * self.ncell and lam_bext.numel() == 3
        fn = self.lib.pic_adjoint_step_record_ordered if ordered else self.lib.pic_adjoint_step_record
        self._check(fn(
            self.ctx, ctypes.c_void_p(record.data_ptr()), record.numel(),
            ctypes.c_void_p(lam_fields.data_ptr()), px, pw, ctypes.c_void_p(lam_bext.data_ptr()),
            _stream()))

    def adjoint_step(self, lam_fields: torch.Tensor, lam_x: list, lam_w: list, lam_bext: torch.Tensor):
        """One reverse step (include/pic.h): the context holds the state the
        step was taken from; lam_* hold the adjoint of the state after it and
        are replaced by the adjoint of the state before it.  lam_x[s] and
        lam_w[s] are (3, count) FP64 device tensors in particle-id order (None
        for immobile species); lam_bext (3,) accumulates dL/dB_ext."""
        px, pw = self._lam_ptrs(lam_x, lam_w)
        assert lam_fields.numel() == 6 * self.ncell and lam_bext.numel() == 3
        self._check(self.lib.pic_adjoint_step(
            self.ctx, ctypes.c_void_p(lam_fields.data_ptr()), px, pw,
            ctypes.c_void_p(lam_bext.data_ptr()), _stream()))

    # -- fields ----------------------------------------------------------
    def aux_line(self) -> np.ndarray:
        """The source's auxiliary line (E^y then B^z, PIC_AUX each) from the workspace."""
        torch.cuda.synchronize()
        sz = L.Sizes()
        L.check(self.lib.pic_query_sizes(ctypes.byref(self.desc), 0, ctypes.byref(sz)))
        nbytes = 2 * L.PIC_AUX * 8
        raw = self.workspace[sz.workspace_bytes - _align(nbytes):][:nbytes]
        return raw.view(torch.float64).cpu().numpy()

    @property
    def fields(self) -> torch.Tensor:
        """(9, nz, ny, nx) view: Ex Ey Ez Bx By Bz Jx Jy Jz."""
        return self.fields_t.view((9,) + self.shape)

    def fields_numpy(self) -> np.ndarray:
        torch.cuda.synchronize()
        return self.fields.cpu().numpy()
