"""CPU oracle for GP population evaluation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``gp_oracle.c`` (plain C,
binary64 accumulation) through ctypes and shares nothing with the HIP
evaluator.  See the header of ``gp_oracle.c`` for what is computed and which
reading of the paper each operator follows.

Pinned against the paper and against closed forms in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gp_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

SUM_ABS, MSE, HITS, CASES, CLASS_ERR = 0, 1, 2, 3, 4
_KINDS = {"sum_abs": SUM_ABS, "mse": MSE, "hits": HITS, "cases": CASES, "class_err": CLASS_ERR}
_INT_KINDS = (HITS, CLASS_ERR)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fno-builtin", "-fPIC", "-shared", "-pthread", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class LgpIns(C.Structure):
    _fields_ = [("op", C.c_int32), ("n_args", C.c_int32), ("kind", C.c_int32 * 2),
                ("feat", C.c_int32 * 2), ("cval", C.c_float * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_tree_outputs.argtypes = [P, P, P, C.c_int32, P, C.c_int32, C.c_int64, C.c_int, P]
        L.orc_linear_outputs.argtypes = [P, P, P, P, C.c_int32, C.c_int32, P, C.c_int32, C.c_int64, C.c_int, P]
        L.orc_fitness.argtypes = [P, P, C.c_int64, C.c_int, P, P, P]
        L.orc_eval_tree.argtypes = [P, P, P, C.c_int32, P, C.c_int32, C.c_int64, P, C.c_int, C.c_int, C.c_int, P, P]
        L.orc_eval_linear.argtypes = [P, P, P, P, C.c_int32, C.c_int32, P, C.c_int32, C.c_int64, P, C.c_int, C.c_int, C.c_int, P, P]
        L.orc_prefix_to_rpn.argtypes = [P, P, C.c_int64, P, P]
        L.orc_rpn_eval.argtypes = [P, P, C.c_int64, P, C.c_int64, C.c_int64, P, P, P]
        L.orc_rpn_to_lgp.argtypes = [P, P, C.c_int64, P, P]
        L.orc_lgp_eval.argtypes = [P, C.c_int64, P, C.c_int64, C.c_int64, P, P, P]
        L.orc_bool_outputs.argtypes = [P, P, C.c_int32, P, C.c_int32, C.c_int64, P]
        L.orc_bool_hits.argtypes = [P, P, C.c_int32, P, C.c_int32, C.c_int64, P, P]
        L.orc_apply.argtypes = [C.c_int, C.c_float, C.c_float]
        L.orc_apply.restype = C.c_float
        L.orc_apply3.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float]
        L.orc_apply3.restype = C.c_float
        assert L.orc_sizeof_lgp_ins() == C.sizeof(LgpIns)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def kind_id(kind) -> int:
    return _KINDS[kind] if isinstance(kind, str) else int(kind)


# ---------------------------------------------------------------------------
def tree_outputs(tok, cst, off, X, nudge=0):
    """Per-case outputs o[p, c] of prefix trees (recursive interpreter)."""
    tok, cst, off, X = _c(tok, np.int32), _c(cst, np.float32), _c(off, np.int64), _c(X, np.float32)
    F, N = X.shape
    P = len(off) - 1
    out = np.empty((P, N), np.float32)
    rc = lib().orc_tree_outputs(_p(tok), _p(cst), _p(off), P, _p(X), F, N, nudge, _p(out))
    if rc != 0:
        raise ValueError("oracle: malformed tree program")
    return out


def linear_outputs(code, off, cst, cst_off, n_reg, X, nudge=0):
    code, off = _c(code, np.uint32), _c(off, np.int64)
    cst, cst_off, X = _c(cst, np.float32), _c(cst_off, np.int64), _c(X, np.float32)
    F, N = X.shape
    P = len(off) - 1
    out = np.empty((P, N), np.float32)
    rc = lib().orc_linear_outputs(_p(code), _p(off), _p(cst), _p(cst_off), P, n_reg,
                                  _p(X), F, N, nudge, _p(out))
    if rc != 0:
        raise ValueError("oracle: malformed linear program")
    return out


def fitness(o, y, kind):
    o, y = _c(o, np.float32), _c(y, np.float32)
    s = C.c_double(); f = C.c_float(); h = C.c_int32()
    rc = lib().orc_fitness(_p(o), _p(y), len(o), kind_id(kind), C.byref(s), C.byref(f), C.byref(h))
    if rc != 0:
        raise ValueError("oracle: bad fitness kind")
    return (h.value if kind_id(kind) in _INT_KINDS else f.value), s.value


def eval_tree(tok, cst, off, X, y, kind, nudge=0, threads=1, return_sums=False):
    tok, cst, off, X = _c(tok, np.int32), _c(cst, np.float32), _c(off, np.int64), _c(X, np.float32)
    F, N = X.shape
    P = len(off) - 1
    k = kind_id(kind)
    y = _c(y if y is not None else np.zeros(N, np.float32), np.float32)
    out = np.empty((P, N) if k == CASES else P, np.int32 if k in _INT_KINDS else np.float32)
    sums = np.zeros(P, np.float64)
    rc = lib().orc_eval_tree(_p(tok), _p(cst), _p(off), P, _p(X), F, N, _p(y), k, nudge,
                             threads, _p(out), _p(sums))
    if rc != 0:
        raise ValueError("oracle: malformed input")
    return (out, sums) if return_sums else out


def eval_linear(code, off, cst, cst_off, n_reg, X, y, kind, nudge=0, threads=1, return_sums=False):
    code, off = _c(code, np.uint32), _c(off, np.int64)
    cst, cst_off, X = _c(cst, np.float32), _c(cst_off, np.int64), _c(X, np.float32)
    F, N = X.shape
    P = len(off) - 1
    k = kind_id(kind)
    y = _c(y if y is not None else np.zeros(N, np.float32), np.float32)
    out = np.empty((P, N) if k == CASES else P, np.int32 if k in _INT_KINDS else np.float32)
    sums = np.zeros(P, np.float64)
    rc = lib().orc_eval_linear(_p(code), _p(off), _p(cst), _p(cst_off), P, n_reg, _p(X), F, N,
                               _p(y), k, nudge, threads, _p(out), _p(sums))
    if rc != 0:
        raise ValueError("oracle: malformed input")
    return (out, sums) if return_sums else out


def apply(op, a, b=0.0):
    return np.float32(lib().orc_apply(op, float(np.float32(a)), float(np.float32(b))))


def apply3(op, a, b, c):
    """A three-operand function (IF) on one case."""
    return np.float32(lib().orc_apply3(op, float(np.float32(a)), float(np.float32(b)), float(np.float32(c))))


def apply_vec(op, a, b=None):
    a = np.asarray(a, np.float32)
    b = np.zeros_like(a) if b is None else np.asarray(b, np.float32)
    f = lib().orc_apply
    return np.array([f(op, float(x), float(z)) for x, z in zip(a, b)], np.float32)


# ---------------------------------------------------------------------------
# The paper's representations
# ---------------------------------------------------------------------------
def prefix_to_rpn(tok, cst):
    tok, cst = _c(tok, np.int32), _c(cst, np.float32)
    ot = np.empty_like(tok); oc = np.empty_like(cst)
    if lib().orc_prefix_to_rpn(_p(tok), _p(cst), len(tok), _p(ot), _p(oc)) != 0:
        raise ValueError("oracle: malformed tree")
    return ot, oc


def rpn_eval(tok, cst, X, c):
    tok, cst, X = _c(tok, np.int32), _c(cst, np.float32), _c(X, np.float32)
    r = C.c_float(); d = C.c_int32(); f = C.c_int32()
    if lib().orc_rpn_eval(_p(tok), _p(cst), len(tok), _p(X), X.shape[1], c,
                          C.byref(r), C.byref(d), C.byref(f)) != 0:
        raise ValueError("oracle: malformed rpn")
    return np.float32(r.value), d.value, f.value


def rpn_to_lgp(tok, cst):
    tok, cst = _c(tok, np.int32), _c(cst, np.float32)
    out = (LgpIns * max(1, len(tok)))()
    m = C.c_int64()
    if lib().orc_rpn_to_lgp(_p(tok), _p(cst), len(tok), out, C.byref(m)) != 0:
        raise ValueError("oracle: malformed rpn")
    return out, m.value


def lgp_eval(ins, m, X, c):
    X = _c(X, np.float32)
    r = C.c_float(); d = C.c_int32(); f = C.c_int32()
    if lib().orc_lgp_eval(ins, m, _p(X), X.shape[1], c, C.byref(r), C.byref(d), C.byref(f)) != 0:
        raise ValueError("oracle: malformed lgp")
    return np.float32(r.value), d.value, f.value


# ---------------------------------------------------------------------------
# Boolean trees over bit-packed cases (bit b of word w is case 32 w + b)
# ---------------------------------------------------------------------------
def bool_outputs(tok, off, Xw):
    """Output words (P, W) of Boolean trees on feature-major words Xw (F, W)."""
    tok, off = _c(tok, np.int32), _c(off, np.int64)
    Xw = _c(Xw, np.uint32)
    F, W = Xw.shape
    P = len(off) - 1
    out = np.zeros((P, W), np.uint32)
    rc = lib().orc_bool_outputs(_p(tok), _p(off), P, _p(Xw), F, W, _p(out))
    if rc != 0:
        raise ValueError("malformed Boolean tree")
    return out


def eval_bool(tok, off, Xw, n_cases, yw):
    """Hit counts (int64[P]) of Boolean trees: cases whose output bit equals
    the target bit, counted case by case."""
    tok, off = _c(tok, np.int32), _c(off, np.int64)
    Xw, yw = _c(Xw, np.uint32), _c(yw, np.uint32)
    F = Xw.shape[0]
    P = len(off) - 1
    hits = np.zeros(P, np.int64)
    rc = lib().orc_bool_hits(_p(tok), _p(off), P, _p(Xw), F, int(n_cases), _p(yw), _p(hits))
    if rc != 0:
        raise ValueError("malformed Boolean tree")
    return hits
