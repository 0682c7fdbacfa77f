"""MI355X (gfx950) GP population evaluator -- thin Python binding.

Every function here marshals arguments and calls the C ABI of ``libgp.so``
(declared in ``include/gp.h``); all evaluation runs in the HIP kernels.
Program arrays are host numpy arrays; case matrices, targets and outputs are
device tensors (torch, used only for device memory and streams) or raw device
pointers.  The library must be built first (``python -m
paper_1601_00221_amd.build``); importing works without it, calling does not.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gp.h")

GP_OK, GP_E_INVAL, GP_E_NOMEM, GP_E_DEPTH, GP_E_DEVICE, GP_E_AGAIN, GP_E_NOTFOUND, GP_E_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
GP_FIT_SUM_ABS, GP_FIT_MSE, GP_FIT_HITS, GP_OUT_CASES = 0, 1, 2, 3
KINDS = {"sum_abs": 0, "mse": 1, "hits": 2, "cases": 3}
STATUS_NAMES = {0: "GP_OK", -1: "GP_E_INVAL", -2: "GP_E_NOMEM", -3: "GP_E_DEPTH",
                -4: "GP_E_DEVICE", -5: "GP_E_AGAIN", -6: "GP_E_NOTFOUND", -7: "GP_E_TIMEOUT"}


class GPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class LowerStats(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_instr", C.c_int32), ("max_depth", C.c_int32),
                ("stack_fetches", C.c_int32), ("n_values", C.c_int32), ("n_reversed", C.c_int32)]


class ProgsetInfo(C.Structure):
    _fields_ = [("n_prog", C.c_int32), ("form", C.c_int32), ("n_feat", C.c_int32),
                ("max_depth", C.c_int32), ("n_instr", C.c_int64), ("n_gpop", C.c_int64)]


_lib = None


def lib():
    """Load libgp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgp.so is not built: run `python -m paper_1601_00221_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "gp_eval_tree": [P, P, P, i32, P, i32, i64, P, i32, P, P],
            "gp_eval_linear": [P, P, P, P, i32, i32, P, i32, i64, P, i32, P, P],
            "gp_progset_tree": [P, P, P, i32, i32, P, P],
            "gp_progset_linear": [P, P, P, P, i32, i32, i32, P, P],
            "gp_progset_eval": [P, P, i32, i64, P, i32, P, P],
            "gp_progset_get_info": [P, P],
            "gp_progset_destroy": [P],
            "gp_lower_tree": [P, P, i64, i32, P, i64, P],
            "gp_timing_enable": [C.c_int],
            "gp_timing_read": [P, P, C.c_int],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gp_last_error.restype = C.c_char_p
        L.gp_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != GP_OK:
        raise GPError(rc, lib().gp_last_error().decode())


def last_error() -> str:
    return lib().gp_last_error().decode()


def version() -> str:
    return lib().gp_version().decode()


def _np(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data_as(C.c_void_p)


def dptr(t):
    """Device pointer of a torch tensor (or an int address / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return C.c_void_p(t)
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def stream_ptr(stream=None):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def kind_id(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


# ---------------------------------------------------------------------------
# One-shot evaluation
# ---------------------------------------------------------------------------
def gp_eval_tree(tok, cst, off, X, y, kind, out, n_feat=None, stream=None):
    """X: (F, N) float32 device tensor; y: (N,) float32 device tensor (None for
    kind "cases"); out: device tensor float32[P] / int32[P] / float32[P, N]."""
    tok, tp = _np(tok, np.int32)
    cst, cp = _np(cst, np.float32)
    off, op = _np(off, np.int64)
    F, N = int(X.shape[0]), int(X.shape[1])
    check(lib().gp_eval_tree(tp, cp, op, len(off) - 1, dptr(X), n_feat or F, N, dptr(y),
                             kind_id(kind), dptr(out), stream_ptr(stream)))


def gp_eval_linear(code, off, cst, cst_off, n_reg, X, y, kind, out, n_feat=None, stream=None):
    code, kp = _np(code, np.uint32)
    off, op = _np(off, np.int64)
    cst, cp = _np(cst if cst is not None else np.zeros(0), np.float32)
    cst_off, cop = _np(cst_off if cst_off is not None else np.zeros(len(off), np.int64), np.int64)
    F, N = int(X.shape[0]), int(X.shape[1])
    check(lib().gp_eval_linear(kp, op, cp, cop, len(off) - 1, n_reg, dptr(X), n_feat or F, N,
                               dptr(y), kind_id(kind), dptr(out), stream_ptr(stream)))


# ---------------------------------------------------------------------------
# Resident program sets
# ---------------------------------------------------------------------------
class ProgSet:
    """Programs lowered and uploaded once (gp_progset_*)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def tree(cls, tok, cst, off, n_feat, stream=None):
        tok, tp = _np(tok, np.int32)
        cst, cp = _np(cst, np.float32)
        off, op = _np(off, np.int64)
        h = C.c_void_p()
        check(lib().gp_progset_tree(tp, cp, op, len(off) - 1, n_feat, stream_ptr(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def linear(cls, code, off, cst, cst_off, n_reg, n_feat, stream=None):
        code, kp = _np(code, np.uint32)
        off, op = _np(off, np.int64)
        cst, cp = _np(cst if cst is not None else np.zeros(0), np.float32)
        cst_off, cop = _np(cst_off if cst_off is not None else np.zeros(len(off), np.int64), np.int64)
        h = C.c_void_p()
        check(lib().gp_progset_linear(kp, op, cp, cop, len(off) - 1, n_reg, n_feat, stream_ptr(stream),
                                      C.byref(h)))
        return cls(h)

    def eval(self, X, y, kind, out, stream=None):
        check(lib().gp_progset_eval(self._h, dptr(X), int(X.shape[0]), int(X.shape[1]), dptr(y),
                                    kind_id(kind), dptr(out), stream_ptr(stream)))

    def info(self) -> dict:
        i = ProgsetInfo()
        check(lib().gp_progset_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in ProgsetInfo._fields_}

    def close(self):
        if self._h:
            check(lib().gp_progset_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Host lowering (no GPU needed)
# ---------------------------------------------------------------------------
def gp_lower_tree(tok, cst, n_feat):
    """Returns (words uint32[2*n_instr], stats dict)."""
    tok, tp = _np(tok, np.int32)
    cst, cp = _np(cst, np.float32)
    words = np.zeros(2 * max(1, len(tok)), np.uint32)
    st = LowerStats()
    check(lib().gp_lower_tree(tp, cp, len(tok), n_feat, words.ctypes.data_as(C.c_void_p), len(words),
                              C.byref(st)))
    stats = {k: getattr(st, k) for k, _ in LowerStats._fields_}
    return words[:2 * stats["n_instr"]], stats


def timing_enable(on: bool = True):
    check(lib().gp_timing_enable(1 if on else 0))


def timing_read(reset: bool = True):
    """(launches, total_ms) of the evaluation kernels since the last reset."""
    n = C.c_int64()
    ms = C.c_double()
    check(lib().gp_timing_read(C.byref(n), C.byref(ms), 1 if reset else 0))
    return n.value, ms.value


def out_tensor(kind, n_prog, n_cases, device="cuda"):
    import torch
    k = kind_id(kind)
    if k == GP_FIT_HITS:
        return torch.empty(n_prog, dtype=torch.int32, device=device)
    if k == GP_OUT_CASES:
        return torch.empty((n_prog, n_cases), dtype=torch.float32, device=device)
    return torch.empty(n_prog, dtype=torch.float32, device=device)
