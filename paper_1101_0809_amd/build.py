"""Build the gfx950 shared library ``libpic.so`` from ``csrc/*.hip`` with hipcc.

Run as ``python -m paper_1101_0809_amd.build`` (or call :func:`build`).  Every
HIP source is compiled for gfx950 only and linked into one shared library next
to this file.

Packed FP32 arithmetic (the v_pk_add/mul/fma_f32 instructions) is kept out of
the device code: ``-Xclang -target-feature -Xclang -packed-fp32-ops`` removes
the feature from the gfx950 compilation.  hipcc passes the flag to the host
compilation too, where x86 has no such feature: that pass prints "not a
recognized feature for this target (ignoring feature)", which is filtered from
the build output.  After compiling, the build extracts each object's gfx950
code object and disassembles it; any packed FP32 instruction fails the build.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


PACKED_FP32 = ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32")
HOST_FLAG_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def llvm_tool(name: str) -> str:
    for d in (os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin"),
              "/opt/rocm/llvm/bin", "/opt/rocm/lib/llvm/bin"):
        p = os.path.join(d, name)
        if os.path.exists(p):
            return p
    raise RuntimeError(f"{name} not found; the build check needs the ROCm LLVM tools")


def packed_fp32_count(obj: str, tmp: str) -> int:
    """Packed FP32 instructions in the gfx950 code object of a hipcc object file."""
    fatbin = obj + ".fatbin"
    code = obj + ".gfx950"
    subprocess.check_call([llvm_tool("llvm-objcopy"), f"--dump-section=.hip_fatbin={fatbin}", obj, os.devnull])
    subprocess.check_call([llvm_tool("clang-offload-bundler"), "--type=o", f"--input={fatbin}",
                           f"--output={code}", f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}", "--unbundle"])
    text = subprocess.run([llvm_tool("llvm-objdump"), "-d", code], check=True, capture_output=True,
                          text=True).stdout
    return sum(text.count(op) for op in PACKED_FP32)


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the GPU library needs ROCm")
    return path


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every csrc/*.hip to an object and link libpic.so (always rebuilds)."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="picbuild") as tmp:
        procs = []
        objs = []
        for s in srcs:
            o = os.path.join(tmp, os.path.basename(s) + ".o")
            objs.append(o)
            cmd = [cc, *HIP_FLAGS, "-c", s, "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            if len(procs) >= jobs:
                _wait(procs.pop(0))
        for p in procs:
            _wait(p)
        for s, o in zip(srcs, objs):
            k = packed_fp32_count(o, tmp)
            if k:
                raise RuntimeError(f"{os.path.basename(s)}: {k} packed FP32 instructions in the gfx950 code")
        tmp_lib = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp_lib, LIB)
    return LIB


def _wait(item):
    src, proc = item
    out, _ = proc.communicate()
    text = out.decode(errors="replace")
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{text}")
    text = "\n".join(l for l in text.splitlines() if HOST_FLAG_NOTE not in l)
    if text.strip():
        sys.stderr.write(text + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
