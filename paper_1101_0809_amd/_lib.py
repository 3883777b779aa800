"""ctypes binding of the C ABI in ``include/pic.h`` (argument marshalling only).

The shared library ``libpic.so`` is built in-tree by
``paper_1101_0809_amd.build``; loading fails loudly if it is missing, there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ERANGE, PIC_ECFL, PIC_EDEVICE, PIC_ESTATE, PIC_ESIZE = 0, -1, -2, -3, -4, -5, -6
PIC_FP64, PIC_FP32C = 0, 1
PIC_B_HALF, PIC_E_FULL = 1, 2
PIC_AUX = 8192  # source line length (include/pic.h)

# Every symbol include/pic.h declares (checked by the CPU tests).
EXPORTS = (
    "pic_query_sizes", "pic_init_grid", "pic_add_species", "pic_load_particles", "pic_step",
    "pic_deposit_J", "pic_field_solve", "pic_diagnostics", "pic_diagnostics_static",
    "pic_particle_count",
    "pic_get_particles", "pic_sort", "pic_last_fallback_fraction", "pic_last_migrant_fraction",
    "pic_timing_start",
    "pic_timing_stop", "pic_get_host_state", "pic_set_host_state", "pic_destroy",
    "pic_adjoint_seed_field_energy", "pic_adjoint_step", "pic_adjoint_record_bytes",
    "pic_adjoint_record", "pic_adjoint_step_record", "pic_adjoint_step_record_ordered",
    "pic_adjoint_reorder", "pic_solve_poisson", "pic_set_vector_potential",
    "pic_get_vector_potential",
    "pic_last_error", "pic_version",
)


class GridDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("sort_every", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("dt", ctypes.c_double), ("c", ctypes.c_double), ("bext", ctypes.c_double * 3),
                ("src_kind", ctypes.c_int32), ("src_plane", ctypes.c_int32),
                ("src_amp", ctypes.c_double), ("src_omega", ctypes.c_double),
                ("src_ramp", ctypes.c_double), ("field_form", ctypes.c_int32),
                ("xbc", ctypes.c_int32)]


class SpeciesDesc(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("mobile", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("capacity", ctypes.c_int64)]


class Sizes(ctypes.Structure):
    _fields_ = [("field_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("particle_bytes", ctypes.c_size_t)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_particles", ctypes.c_int64),
                ("kinetic", ctypes.c_double), ("field_e", ctypes.c_double),
                ("field_b", ctypes.c_double), ("charge", ctypes.c_double),
                ("gauss_abs", ctypes.c_double), ("gauss_rel", ctypes.c_double),
                ("rho_mobile_max", ctypes.c_double), ("divb_max", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("kinetic_half_step", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class HostState(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("since_sort", ctypes.c_int32),
                ("r0_valid", ctypes.c_int32), ("nsp", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n", ctypes.c_int64 * 4), ("sorted", ctypes.c_int32 * 4),
                ("copy", ctypes.c_int32 * 4)]


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pic error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libpic.so and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # load it first so that this library binds to it and can take torch's
    # streams and allocations.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1101_0809_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sigs = {
        "pic_query_sizes": (I, [ctypes.POINTER(GridDesc), I64, ctypes.POINTER(Sizes)]),
        "pic_init_grid": (I, [ctypes.POINTER(GridDesc), P, ctypes.c_size_t, P, ctypes.c_size_t,
                              ctypes.POINTER(P)]),
        "pic_add_species": (I, [P, ctypes.POINTER(SpeciesDesc), P, ctypes.c_size_t,
                                ctypes.POINTER(I)]),
        "pic_load_particles": (I, [P, I, I64, P, P, P, P]),
        "pic_step": (I, [P, I, P]),
        "pic_deposit_J": (I, [P, P, P, P, I64, P, P]),
        "pic_field_solve": (I, [P, I, P]),
        "pic_diagnostics": (I, [P, ctypes.POINTER(Diag), P]),
        "pic_diagnostics_static": (I, [P, ctypes.POINTER(Diag), P]),
        "pic_particle_count": (I64, [P, I]),
        "pic_get_particles": (I, [P, I, P, P, P, P, P]),
        "pic_sort": (I, [P, P]),
        "pic_last_fallback_fraction": (D, [P, P]),
        "pic_last_migrant_fraction": (D, [P, P]),
        "pic_timing_start": (I, [P, I]),
        "pic_timing_stop": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]),
        "pic_get_host_state": (I, [P, ctypes.POINTER(HostState)]),
        "pic_set_host_state": (I, [P, ctypes.POINTER(HostState)]),
        "pic_adjoint_seed_field_energy": (I, [P, P, P]),
        "pic_adjoint_step": (I, [P, P, ctypes.POINTER(P), ctypes.POINTER(P), P, P]),
        "pic_adjoint_record_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "pic_adjoint_record": (I, [P, P, ctypes.c_size_t, P]),
        "pic_adjoint_step_record": (I, [P, P, ctypes.c_size_t, P, ctypes.POINTER(P), ctypes.POINTER(P),
                                        P, P]),
        "pic_adjoint_step_record_ordered": (I, [P, P, ctypes.c_size_t, P, ctypes.POINTER(P),
                                                ctypes.POINTER(P), P, P]),
        "pic_adjoint_reorder": (I, [P, P, P, ctypes.c_size_t, ctypes.POINTER(P), ctypes.POINTER(P),
                                    ctypes.POINTER(P), ctypes.POINTER(P), P]),
        "pic_solve_poisson": (I, [P, I, D, ctypes.POINTER(I64), ctypes.POINTER(D), P]),
        "pic_set_vector_potential": (I, [P, P, P]),
        "pic_get_vector_potential": (I, [P, P, P]),
        "pic_destroy": (None, [P]),
        "pic_last_error": (ctypes.c_char_p, [P]),
        "pic_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, ctx=None):
    if rc != PIC_OK:
        msg = load().pic_last_error(ctx)
        raise PicError(rc, msg.decode() if msg else "")
