"""CPU checks of the C ABI: the library loads, exports every symbol that
include/pic.h declares, and validates descriptions before touching the GPU.
No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _lib():
    from paper_1101_0809_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libpic.so not built (run python -m paper_1101_0809_amd.build)")
    return L, L.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("pic_init_grid", "pic_load_particles", "pic_step", "pic_deposit_J",
                     "pic_field_solve", "pic_diagnostics"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    names = declared_symbols()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L.EXPORTS)


def _desc(L, **kw):
    d = L.GridDesc()
    d.dims, d.nx, d.ny, d.nz = 3, 16, 16, 16
    d.precision, d.order, d.sort_every, d.interp = L.PIC_FP64, 1, 10, 0
    d.dx = d.dy = d.dz = 1.0
    d.dt, d.c = 0.45, 1.0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_query_sizes():
    L, lib = _lib()
    sz = L.Sizes()
    assert lib.pic_query_sizes(ctypes.byref(_desc(L)), 1000, ctypes.byref(sz)) == 0
    assert sz.field_bytes == 9 * 16 ** 3 * 8
    # two FP64 copies of 8 arrays (1000 elements, 256-byte aligned) + keys/ranks + tiles
    assert sz.particle_bytes >= 2 * 8 * 8 * 1000 + 2 * 4 * 1000
    sz32 = L.Sizes()
    assert lib.pic_query_sizes(ctypes.byref(_desc(L, precision=L.PIC_FP32C)), 1000,
                               ctypes.byref(sz32)) == 0
    assert sz32.particle_bytes < sz.particle_bytes


@pytest.mark.parametrize("kw,code", [
    (dict(dt=0.6), -3),                      # 3 * 0.36 >= 1: Courant limit
    (dict(dt=1.0, nz=1, dims=2), -3),        # c dt / dx = 1
    (dict(dims=2), -1),                      # 2D needs nz == 1
    (dict(dims=4), -1),
    (dict(nx=0), -1),
    (dict(order=3), -1),
    (dict(order=2, precision=1), -1),        # order 2 1/2 is FP64 only
    (dict(precision=7), -1),
    (dict(interp=2), -1),
    (dict(interp=1, order=2), -1),          # conventional: order 1 only
    (dict(interp=1, precision=1), -1),      # conventional: FP64 only
    (dict(precision=1, nx=4096), -1),        # FP32 cell packing limit
    (dict(precision=1, nx=2049), -1),        # 11 bits for the x cell
    (dict(precision=1, ny=2049), -1),        # 11 bits for the y cell
    (dict(precision=1, nz=1025), -1),        # 10 bits for the z cell
    (dict(dx=-1.0), -1),
    (dict(xbc=2), -1),                      # x boundary: 0 periodic, 1 open
    (dict(xbc=1, nx=7), -1),                # open x needs nx >= 8
    (dict(xbc=1, order=2), -1),             # open x: order 1 1/2 only
    (dict(xbc=1, interp=1), -1),
    (dict(xbc=1, field_form=1), -1),        # open x: B carried
    (dict(xbc=1, src_kind=1, src_plane=14), -1),  # source plane <= nx - 3
])
def test_invalid_descriptions_rejected(kw, code):
    L, lib = _lib()
    sz = L.Sizes()
    rc = lib.pic_query_sizes(ctypes.byref(_desc(L, **kw)), 10, ctypes.byref(sz))
    assert rc == code
    assert lib.pic_last_error(None)
    ctx = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(16)
    rc2 = lib.pic_init_grid(ctypes.byref(_desc(L, **kw)), ctypes.cast(buf, ctypes.c_void_p), 16,
                            ctypes.cast(buf, ctypes.c_void_p), 16, ctypes.byref(ctx))
    assert rc2 == code and not ctx.value


@pytest.mark.parametrize("kw", [dict(nx=2048), dict(ny=2048), dict(nz=1024)])
def test_fp32_mode_accepts_its_largest_axes(kw):
    """The packed FP32 cell word's limits themselves are accepted."""
    L, lib = _lib()
    sz = L.Sizes()
    assert lib.pic_query_sizes(ctypes.byref(_desc(L, precision=L.PIC_FP32C, **kw)), 10, ctypes.byref(sz)) == 0


@pytest.mark.parametrize("kw", [dict(xbc=1, nx=8), dict(xbc=1, src_kind=1, src_plane=13),
                                dict(xbc=1, precision=1), dict(xbc=1, dims=2, nz=1)])
def test_open_x_descriptions_accepted(kw):
    L, lib = _lib()
    sz = L.Sizes()
    assert lib.pic_query_sizes(ctypes.byref(_desc(L, **kw)), 10, ctypes.byref(sz)) == 0


def test_two_dimensional_courant_ignores_z():
    L, lib = _lib()
    sz = L.Sizes()
    d = _desc(L, dims=2, nz=1, dt=0.6)   # 2 * 0.36 < 1 in 2D
    assert lib.pic_query_sizes(ctypes.byref(d), 10, ctypes.byref(sz)) == 0


def test_init_rejects_small_buffers():
    L, lib = _lib()
    ctx = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(64)
    rc = lib.pic_init_grid(ctypes.byref(_desc(L)), ctypes.cast(buf, ctypes.c_void_p), 64,
                           ctypes.cast(buf, ctypes.c_void_p), 64, ctypes.byref(ctx))
    assert rc == L.PIC_ESIZE


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1101_0809_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pic_oracle" not in text and "liboracle" not in text, f


def test_python_binding_imports_without_gpu():
    import importlib

    mod = importlib.import_module("paper_1101_0809_amd.sim")
    assert hasattr(mod, "Sim")
    import bench  # noqa: F401  (the benchmark module must import cleanly too)
    import __graft_entry__  # noqa: F401


def test_committed_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """bench.py reports the committed HBM traffic only while the recorded hash
    matches the step kernels' sources: a change to any of the three files,
    the kernel file or either header, turns it off."""
    import hashlib
    import json
    import shutil

    import bench

    src = os.path.join(ROOT, "paper_1101_0809_amd", "csrc")
    dst = tmp_path / "paper_1101_0809_amd" / "csrc"
    dst.mkdir(parents=True)
    names = ("particles.hip", "pic_math.h", "pic_internal.h")
    for n in names:
        shutil.copy(os.path.join(src, n), dst / n)

    def digest():
        h = hashlib.sha256()
        for n in names:
            h.update((dst / n).read_bytes())
        return h.hexdigest()[:16]

    (tmp_path / "profiles").mkdir()
    info = {"source_sha256_16": digest(), "traffic": {"fp32c": 123, "fp64": 456}}
    (tmp_path / "profiles" / "k_particle_step_w.md").write_text(f"x\n<!-- traffic-json {json.dumps(info)} -->\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fp32c", "w") == 123
    assert bench.measured_traffic("fp64", "w") == 456
    assert bench.measured_traffic("fp32c", "other") is None
    for n in names:
        before = (dst / n).read_bytes()
        (dst / n).write_bytes(before + b"\n")
        assert bench.measured_traffic("fp32c", "w") is None, n
        (dst / n).write_bytes(before)
    assert bench.measured_traffic("fp32c", "w") == 123
