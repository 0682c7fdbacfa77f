"""Build libgp.so (HIP for gfx950) in-tree.

    python -m paper_1601_00221_amd.build

Every source is compiled with hipcc for gfx950 only, without floating-point
contraction and without packed FP32 instructions, then linked into
``paper_1601_00221_amd/libgp.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libgp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["lower.cpp", "runtime.cpp", "batch.cpp", "serve.cpp", "core_host.cpp", "core_kernels.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "--offload-arch=gfx950",
    "-ffp-contract=off",
    # packed FP32 (v_pk_*_f32) stays off; the flag is for the device pass only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-inline-asm",   # the core names the VGPRs it owns, which the compiler reserves
]

# The core owns v[NCV ...]; the compiler must never allocate them.  The kernel
# attribute that caps the compiler's VGPRs is checked by compiling the core
# with inline-asm warnings on: every clobbered VGPR the core owns must be
# reported as reserved.
import re


def _check_reserved(src: str):
    sys.path.insert(0, CSRC)
    try:
        import gen_core
    finally:
        sys.path.pop(0)
    flags = [f for f in FLAGS if f != "-Wno-inline-asm"]
    cmd = [HIPCC, *flags, "-I", GEN, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o",
           os.path.join(BUILD, os.path.splitext(src)[0] + "-gfx950.s")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr))
    reserved = set()
    for m in re.finditer(r"clobber list contains reserved registers: ([^\[]*)", r.stderr):
        reserved.update(x.strip() for x in m.group(1).split(","))
    for t, d, nf, ncv in gen_core.VARIANTS:
        end = ncv + max(gen_core.LIN_REGS, d) * t + nf * t
        missing = [n for n in range(ncv, end) if "v%d" % n not in reserved]
        if missing:
            raise RuntimeError("the compiler may allocate core VGPRs %s (variant %s)" % (missing[:8], (t, d, nf, ncv)))


def _stale(src: str, obj: str) -> bool:
    """True if obj is older than src, any header, or the generated core."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.join(GEN, "core_gen.inc"), os.path.abspath(__file__),
            os.path.join(os.path.dirname(PKG), "include", "gp.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *FLAGS, "-I", GEN, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those older than their
    inputs, for development) and link libgp.so."""
    os.makedirs(BUILD, exist_ok=True)
    # generate the hand-written interpreter core for every kernel variant
    sys.path.insert(0, CSRC)
    try:
        import gen_core
    finally:
        sys.path.pop(0)
    inc = os.path.join(GEN, "core_gen.inc")
    old = open(inc).read() if os.path.exists(inc) else None
    if incremental and old is not None:
        tmp = GEN + ".tmp"
        gen_core.main(tmp)
        new = open(os.path.join(tmp, "core_gen.inc")).read()
        if new != old:
            gen_core.main(GEN)
        shutil.rmtree(tmp, ignore_errors=True)
    else:
        gen_core.main(GEN)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + 1)) as ex:
        check = None
        if not incremental or _stale("core_kernels.hip", os.path.join(BUILD, "core_kernels.o")):
            check = ex.submit(_check_reserved, "core_kernels.hip")
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
        if check is not None:
            check.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
