"""The library's host code (validation, lowering, translation, the
server's scheduler in dry-run mode, GP breeding) and the oracle, built with
the address and undefined-behaviour sanitizers and run on random and
malformed input on the CPU (no device code: the kernel launchers are
stand-ins that report no device)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1601_00221_amd", "csrc")
HOST_SOURCES = ["lower.cpp", "runtime.cpp", "batch.cpp", "serve.cpp", "core_host.cpp", "evolve.cpp", "blockgp.cpp"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h") or _runtime("libasan.so") is None,
                    reason="needs the HIP headers and the gcc sanitizer runtimes")
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    sys.path.insert(0, CSRC)
    import gen_core
    gen = tmp_path / "gen"
    gen_core.main(str(gen))          # the generated handler tables the host code includes
    objs = []
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-D__device__=",
             "-D__forceinline__=inline", "-I/opt/rocm/include", "-I" + str(gen), "-I" + CSRC, "-I" + os.path.join(ROOT, "include")] + SAN
    for src in HOST_SOURCES + [os.path.join(HERE, "native", "launch_stubs.cpp")]:
        o = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run(["g++", *flags, "-c", os.path.join(CSRC, src) if "/" not in src else src, "-o", str(o)],
                       check=True)
        objs.append(str(o))
    lib = tmp_path / "libgp_san.so"
    subprocess.run(["g++", "-shared", *SAN, "-o", str(lib), *objs, "-L/opt/rocm/lib", "-lamdhip64", "-lpthread"],
                   check=True)
    orc = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin", "-fPIC",
                    "-shared", "-pthread", *SAN, os.path.join(ROOT, "oracle", "gp_oracle.c"), "-o", str(orc), "-lm"],
                   check=True)
    env = dict(os.environ)
    pre = [_runtime("libasan.so"), _runtime("libubsan.so")]
    env["LD_PRELOAD"] = " ".join([p for p in pre if p] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    r = subprocess.run([sys.executable, os.path.join(HERE, "native", "sanitize_exercise.py"), str(lib), str(orc)],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized host paths: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-4000:]
