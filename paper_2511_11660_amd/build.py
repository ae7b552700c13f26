"""Build steps for the native parts, run by ``__graft_entry__.build()``.

  libsta.so        HIP kernels + host runtime (hipcc, gfx950), the product
  libstasynth.so   seeded design generator (gcc)
  liboracle.so     FP64 CPU oracle used by tests only (gcc)

Everything is built in-tree so the shared objects travel with the sources.
"""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBSTA = os.path.join(PKG, "libsta.so")
LIBSYNTH = os.path.join(PKG, "synth", "libstasynth.so")
LIBORACLE = os.path.join(ROOT, "oracle", "liboracle.so")

# Packed FP32 instructions are disabled: this codebase writes scalar float
# code and leaves vectorization to the compiler's non-packed forms.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}")


def build_sta() -> str:
    """Compiles the kernels and host runtime, then links the shared object
    without a hard dependency on one HIP runtime copy: the process supplies it
    (the binding preloads the runtime the process already uses, so torch and
    this library share one HIP/HSA runtime, its streams and allocations)."""
    srcs = [os.path.join(CSRC, "sta_kernels.hip"), os.path.join(CSRC, "sta_rc_estimate.hip"),
            os.path.join(CSRC, "sta_host.cpp")]
    objs = []
    bdir = os.path.join(CSRC, "_build")
    os.makedirs(bdir, exist_ok=True)
    compile_flags = [f for f in HIP_FLAGS if f != "-shared"]
    for src in srcs:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        _run([_hipcc(), *compile_flags, "-I", os.path.join(ROOT, "include"), "-x", "hip", "-c", src,
              "-o", obj])
        objs.append(obj)
    tmp = LIBSTA + ".tmp"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clangxx):
        clangxx = shutil.which("clang++") or "g++"
    _run([clangxx, "-shared", "-fPIC", "-o", tmp, *objs, "-Wl,--no-undefined-version"])
    os.replace(tmp, LIBSTA)
    return LIBSTA


def build_synth() -> str:
    tmp = LIBSYNTH + ".tmp"
    _run(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp,
          os.path.join(PKG, "synth", "synth.c"), "-lm"])
    os.replace(tmp, LIBSYNTH)
    return LIBSYNTH


def build_oracle() -> str:
    tmp = LIBORACLE + ".tmp"
    _run(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp,
          os.path.join(ROOT, "oracle", "sta_oracle.c"), "-lm"])
    os.replace(tmp, LIBORACLE)
    return LIBORACLE


def build_all() -> list[str]:
    return [build_synth(), build_oracle(), build_sta()]


if __name__ == "__main__":
    for p in build_all():
        print(p)
