"""The evaluator's sin/cos/exp/log (binary64 evaluation of a binary32
argument, rounded once), compiled for the host, against the oracle's
definition of the same operations: the same binary32 result for all but a
vanishing fraction of arguments, never more than 1 ulp away, and exactly the
oracle's value on special arguments."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def gm(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("gm") / "libgm.so")
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-I", os.path.join(ROOT, "paper_1601_00221_amd", "csrc"),
           os.path.join(HERE, "native", "gp_math_shim.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    lib = C.CDLL(out)
    lib.gm_eval.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int64]
    lib.gm_eval_n8.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int64]

    def run(op, x, batched=False):
        x = np.ascontiguousarray(x, np.float32)
        y = np.empty_like(x)
        if batched:
            n = len(x) // 8 * 8
            lib.gm_eval_n8(op, x.ctypes.data, y.ctypes.data, n)
            lib.gm_eval(op, x[n:].ctypes.data, y[n:].ctypes.data, len(x) - n)
        else:
            lib.gm_eval(op, x.ctypes.data, y.ctypes.data, len(x))
        return y
    return run


def _ulps(a, b):
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    d = np.abs(ia - ib)
    both_nan = np.isnan(a) & np.isnan(b)
    return np.where(both_nan, 0, d)


def _args():
    rng = synth.rng_for(77)
    # random bit patterns over all finite binary32 values, plus dense ranges
    bits = rng.integers(0, 2**32, size=400000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    dense = [rng.uniform(-10, 10, 300000), rng.uniform(-120, 90, 200000), rng.uniform(-1e6, 1e6, 100000),
             rng.uniform(0, 2e-6, 50000), np.arange(-2000, 2000) * (np.pi / 4)]
    special = [0.0, -0.0, 1.0, -1.0, 88.0, 88.5, 1e30, -1e30, 3.4e38, -3.4e38, 1e-6, 9.99999997e-7, 1e-45,
               -1e-45, 524287.9, 524288.0, -524288.0, np.inf, -np.inf, np.nan, 1.5707964, 3.1415927, -104.0,
               -103.97, -103.95, 0.693147, 1.4142135, 0.70710677]
    return np.concatenate([x] + [np.asarray(d, np.float32) for d in dense] + [np.asarray(special, np.float32)])


@pytest.mark.parametrize("op", [synth.SIN, synth.COS, synth.EXPC, synth.PLOG])
def test_transcendental_matches_oracle(gm, op):
    x = _args()
    got = gm(op, x)
    ref = np.array([oracle.apply(op, float(v)) for v in x], np.float32)
    d = _ulps(got, ref)
    assert d.max() <= 1, (synth.NAMES[op], x[d > 1][:5], got[d > 1][:5], ref[d > 1][:5])
    assert (d == 0).mean() >= 0.99999, (synth.NAMES[op], (d != 0).sum())
    # special arguments exactly
    sp = x[-28:]
    assert (d[-28:] == 0).all(), (synth.NAMES[op], sp[d[-28:] != 0])


@pytest.mark.parametrize("op", [synth.SIN, synth.COS, synth.EXPC, synth.PLOG])
def test_batched_form_is_identical(gm, op):
    x = _args()
    a = gm(op, x)
    b = gm(op, x, batched=True)
    assert ((a.view(np.int32) == b.view(np.int32)) | (np.isnan(a) & np.isnan(b))).all()


def test_tables_regenerate_from_their_definitions(tmp_path):
    """The committed reduction tables are what the generator computes from
    the mathematical definitions (300-bit mpmath)."""
    import importlib.util
    gen = os.path.join(ROOT, "paper_1601_00221_amd", "csrc", "gen_math_tables.py")
    spec = importlib.util.spec_from_file_location("gen_math_tables", gen)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = mod.main(str(tmp_path))
    with open(out) as f, open(os.path.join(ROOT, "paper_1601_00221_amd", "csrc", "gp_math_tables.h")) as g:
        assert f.read() == g.read()


def test_table_spot_values():
    """Entries against closed forms: sin(pi/4) = cos(pi/4) = 2^-1/2 (j = 16),
    sin(pi/2) = 1 and cos(pi/2) = 0 (j = 32), 2^(32/64) = 2^1/2, the bucket
    centre 1 with c = 1 and -log c = 0, and the chunks of 64/pi summing to
    64/pi."""
    import re
    import mpmath
    text = open(os.path.join(ROOT, "paper_1601_00221_amd", "csrc", "gp_math_tables.h")).read()

    def arr(name):
        body = re.search(name + r"\[\d+\] = \{([^}]*)\}", text).group(1)
        return [float.fromhex(x.strip()) for x in body.split(",") if x.strip()]
    h = float.fromhex("0x1.6a09e667f3bcdp-1")    # nearest binary64 to 2^-1/2
    sc = arr("kSinCos")
    assert len(sc) == 256 and sc[2 * 16] == h and sc[2 * 16 + 1] == h
    assert sc[0] == 0.0 and sc[1] == 1.0 and sc[2 * 32] == 1.0 and sc[2 * 32 + 1] == 0.0 and sc[2 * 64] == 0.0
    assert arr("kExp2J")[32] == float.fromhex("0x1.6a09e667f3bcdp+0")
    k0 = int(re.search(r"GPX_LOG_K0 0x([0-9A-F]+)", text).group(1), 16)
    ct = arr("kLogCT")
    one = 0x3F800000 >> 15      # the bucket whose centre is 1.0
    assert ct[2 * (one - k0)] == 1.0 and ct[2 * (one - k0) + 1] == 0.0
    chunks = arr("kPiChunks")
    mpmath.mp.prec = 300
    total = sum(mpmath.mpf(c) for c in chunks)
    assert abs(total - 64 / mpmath.pi) < mpmath.mpf(2) ** -210
    for c in chunks:     # at most 28 significant bits: exact products with binary32 values
        m, e = mpmath.frexp(mpmath.mpf(c))
        assert (m * 2 ** 28) == int(m * 2 ** 28)
