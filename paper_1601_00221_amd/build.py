"""Build libgp.so (HIP for gfx950) in-tree.

    python -m paper_1601_00221_amd.build [--incremental]

Every source is compiled with hipcc for gfx950 only, without floating-point
contraction and without packed FP32 instructions, then linked into
``paper_1601_00221_amd/libgp.so``.  The evaluation kernel is compiled once
per variant, each in a translation unit that gen_core.py writes, so the
variants build in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libgp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["lower.cpp", "runtime.cpp", "batch.cpp", "serve.cpp", "core_host.cpp", "core_kernels.hip",
           "blockgp.cpp", "blockgp_kernels.hip", "evolve.cpp", "noalloc.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "--offload-arch=gfx950",
    "-ffp-contract=off",
    # packed FP32 (v_pk_*_f32) stays off; the flag is for the device pass only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _gen_core():
    sys.path.insert(0, CSRC)
    try:
        import gen_core
    finally:
        sys.path.pop(0)
    return gen_core


def _stale(src_path: str, obj: str) -> bool:
    """True if obj is older than its source, any header, or the generated core."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src_path, os.path.join(GEN, "core_gen.inc"), os.path.join(GEN, "core_dispatch.inc"),
            os.path.abspath(__file__), os.path.join(os.path.dirname(PKG), "include", "gp.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


def _check_reserved(stderr: str, variant) -> None:
    """The core owns v[NCV ...]: the compiler must never allocate them.  The
    kernel attribute that caps the compiler's VGPRs is checked through the
    compiler's inline-asm warnings: every VGPR the core clobbers must be
    reported as reserved."""
    gen_core = _gen_core()
    t, d, nf, ncv, mode = variant
    reserved = set()
    for m in re.finditer(r"clobber list contains reserved registers: ([^\[\n]*)", stderr):
        reserved.update(x.strip() for x in m.group(1).split(","))
    end = ncv + gen_core.reg_levels(d, mode) * t + nf * t
    missing = [n for n in range(ncv, end) if "v%d" % n not in reserved]
    if missing:
        raise RuntimeError("the compiler may allocate core VGPRs %s (variant %s)" % (missing[:8], variant))


def _compile(src_path: str, incremental: bool, variant=None) -> str:
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src_path))[0] + ".o")
    if incremental and not _stale(src_path, obj):
        return obj
    flags = list(FLAGS)
    if variant is None:
        flags.append("-Wno-inline-asm")
    cmd = [HIPCC, *flags, "-I", GEN, "-I", CSRC, "-c", src_path, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    if variant is not None:
        _check_reserved(r.stderr, variant)
    os.replace(obj + ".tmp", obj)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those older than their
    inputs, for development) and link libgp.so."""
    os.makedirs(BUILD, exist_ok=True)
    gen_core = _gen_core()
    gen_core.main(GEN)   # the hand-written interpreter core of every kernel variant
    jobs = [(os.path.join(CSRC, s), None) for s in SOURCES]
    jobs += [(os.path.join(GEN, f), v) for f, v in zip(gen_core.variant_sources(), gen_core.VARIANTS)]
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], incremental, j[1]), jobs))
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
