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
GP_FIT_SUM_ABS, GP_FIT_MSE, GP_FIT_HITS, GP_OUT_CASES, GP_FIT_CLASS_ERR = 0, 1, 2, 3, 4
KINDS = {"sum_abs": 0, "mse": 1, "hits": 2, "cases": 3, "class_err": 4}
GP_MAX_FEAT, GP_MAX_DEPTH, GP_MAX_LEN = 44, 20, 65536
STATUS_NAMES = {0: "GP_OK", -1: "GP_E_INVAL", -2: "GP_E_NOMEM", -3: "GP_E_DEPTH",
                -4: "GP_E_DEVICE", -5: "GP_E_AGAIN", -6: "GP_E_NOTFOUND", -7: "GP_E_TIMEOUT"}


class GPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class LowerStats(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_instr", C.c_int32), ("max_depth", C.c_int32),
                ("stack_fetches", C.c_int32), ("n_values", C.c_int32), ("n_reversed", C.c_int32)]


class EvolveConfig(C.Structure):
    _fields_ = [("pop_size", C.c_int32), ("generations", C.c_int32), ("max_depth", C.c_int32),
                ("max_size", C.c_int32), ("tournament", C.c_int32), ("p_crossover", C.c_float),
                ("p_mutation", C.c_float), ("init_min_depth", C.c_int32), ("init_max_depth", C.c_int32),
                ("mutation_depth", C.c_int32), ("functions", C.c_uint32), ("p_const", C.c_float),
                ("const_lo", C.c_float), ("const_hi", C.c_float), ("kind", C.c_int32), ("seed", C.c_uint64)]


class EvolveResult(C.Structure):
    _fields_ = [("best_fitness", C.c_double), ("best_generation", C.c_int32), ("best_size", C.c_int32),
                ("generations_run", C.c_int32), ("pad", C.c_int32), ("gp_ops", C.c_int64),
                ("eval_seconds", C.c_double), ("breed_seconds", C.c_double), ("total_seconds", C.c_double)]


def evolve_config(functions, kind="mse", pop_size=1000, generations=50, max_depth=50, max_size=1000,
                  tournament=7, p_crossover=0.95, p_mutation=0.2, init_depth=(2, 6), mutation_depth=4,
                  p_const=0.0, const_range=(-1.0, 1.0), seed=1):
    """A gp_evolve_config; the defaults are the paper's Table 2 parameters.
    functions: opcodes of the function set."""
    mask = 0
    for op in functions:
        mask |= 1 << int(op)
    return EvolveConfig(pop_size, generations, max_depth, max_size, tournament, p_crossover, p_mutation,
                        init_depth[0], init_depth[1], mutation_depth, mask, p_const, const_range[0],
                        const_range[1], kind_id(kind), seed)


def _csr_out(cfg):
    cap = cfg.pop_size * cfg.max_size
    return np.zeros(cap, np.int32), np.zeros(cap, np.float32), np.zeros(cfg.pop_size + 1, np.int64), cap


def init_population(cfg, n_feat):
    """gp_init_population: (tok, cst, off) of the initial population (host only)."""
    tok, cst, off, cap = _csr_out(cfg)
    check(lib().gp_init_population(C.byref(cfg), n_feat, tok.ctypes.data, cst.ctypes.data, off.ctypes.data, cap))
    return tok[:off[-1]], cst[:off[-1]], off


def breed(cfg, tok, cst, off, n_feat, score, seed):
    """gp_breed: the next generation of a population (host only)."""
    tok, tp = _np(tok, np.int32)
    cst, cp = _np(cst, np.float32)
    off, op = _np(off, np.int64)
    score, sp = _np(score, np.float64)
    ot, oc, oo, cap = _csr_out(cfg)
    check(lib().gp_breed(C.byref(cfg), tp, cp, op, n_feat, sp, seed, ot.ctypes.data, oc.ctypes.data,
                         oo.ctypes.data, cap))
    return ot[:oo[-1]], oc[:oo[-1]], oo


def evolve(cfg, X, y, n_cases=None, stream=None):
    """gp_evolve: one GP run; X, y device tensors (float32, or 32-bit words
    for a Boolean function set with n_cases in bits).  Returns a dict with
    the result fields, the best fitness per generation and the best program."""
    n = int(X.shape[1]) if n_cases is None else int(n_cases)
    per_gen = np.zeros(cfg.generations + 1, np.float64)
    bt = np.zeros(cfg.max_size, np.int32)
    bc = np.zeros(cfg.max_size, np.float32)
    r = EvolveResult()
    check(lib().gp_evolve(C.byref(cfg), dptr(X), int(X.shape[0]), n, dptr(y), per_gen.ctypes.data,
                          bt.ctypes.data, bc.ctypes.data, cfg.max_size, C.byref(r), stream_ptr(stream)))
    out = {k: getattr(r, k) for k, _ in EvolveResult._fields_ if k != "pad"}
    out["best_per_generation"] = per_gen[:r.generations_run]
    out["best_tok"], out["best_cst"] = bt[:r.best_size].copy(), bc[:r.best_size].copy()
    return out


class ProgsetInfo(C.Structure):
    _fields_ = [("n_prog", C.c_int32), ("form", C.c_int32), ("n_feat", C.c_int32),
                ("max_depth", C.c_int32), ("n_instr", C.c_int64), ("n_gpop", C.c_int64),
                ("variant", C.c_int32), ("pad", C.c_int32)]


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
            "gp_eval_tree_1d": [P, P, P, i32, P, i32, i64, P, i32, i32, P, P],
            "gp_eval_bool": [P, P, i32, P, i32, i64, P, i32, P, P],
            "gp_evolve": [P, P, i32, i64, P, P, P, P, i32, P, P],
            "gp_init_population": [P, i32, P, P, P, i64],
            "gp_breed": [P, P, P, P, i32, P, C.c_uint64, P, P, P, i64],
            "gp_eval_linear": [P, P, P, P, i32, i32, P, i32, i64, P, i32, P, P],
            "gp_progset_tree": [P, P, P, i32, i32, P, P],
            "gp_progset_linear": [P, P, P, P, i32, i32, i32, P, P],
            "gp_progset_bool": [P, P, i32, i32, P, P],
            "gp_progset_eval": [P, P, i32, i64, P, i32, P, P],
            "gp_progset_eval_noalloc": [P, P, i32, i64, P, i32, P, P],
            "gp_progset_get_info": [P, P],
            "gp_progset_destroy": [P],
            "gp_lower_tree": [P, P, i64, i32, P, i64, P],
            "gp_timing_enable": [C.c_int],
            "gp_timing_read": [P, P, C.c_int],
            "gp_eval_batch": [P, i32, P, i32, P, P],
            "gp_tune_batch": [P, i32, P, i32, i32, P, P, P],
            "gp_variant_info": [i32, P, P, P, P, P],
            "gp_serve_create": [P, P],
            "gp_serve_add_dataset": [P, P, i32, i64, P, P],
            "gp_serve_submit": [P, P, P],
            "gp_serve_poll": [P, C.c_uint64, P],
            "gp_serve_wait": [P, C.c_uint64, i64],
            "gp_serve_cancel": [P, C.c_uint64],
            "gp_serve_release": [P, C.c_uint64],
            "gp_serve_stats": [P, P],
            "gp_serve_destroy": [P],
            "gp_core_lower_tree": [P, P, P, i32, i32, i32, C.c_uint64, P, i64, P, P],
            "gp_core_lower_linear": [P, P, P, P, i32, i32, i32, i32, C.c_uint64, P, i64, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gp_num_variants.restype = C.c_int32
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


def gp_eval_bool(tok, off, X, y, kind, out, n_cases, n_feat=None, stream=None):
    """Boolean trees over bit-packed cases.  X: (F, n_words) int32/uint32
    device tensor (bit b of word w is case 32 w + b); y: (n_words,) device
    tensor or None for kind "cases"; out: int32[P] (hits) or int32[P,
    n_words] (output words)."""
    tok, tp = _np(tok, np.int32)
    off, op = _np(off, np.int64)
    F = int(X.shape[0])
    check(lib().gp_eval_bool(tp, op, len(off) - 1, dptr(X), n_feat or F, int(n_cases), dptr(y), kind_id(kind),
                             dptr(out), stream_ptr(stream)))


GP_1D_FORMS = {"rpn": 0, "lgp": 1}


def gp_eval_tree_1d(tok, cst, off, X, y, kind, out, form="rpn", n_feat=None, stream=None):
    """The one-dimensional-stack comparator: same arguments as gp_eval_tree,
    plus form "rpn" (postfix code) or "lgp" (the stack-operand linear form)."""
    tok, tp = _np(tok, np.int32)
    cst, cp = _np(cst, np.float32)
    off, op = _np(off, np.int64)
    F, N = int(X.shape[0]), int(X.shape[1])
    fid = GP_1D_FORMS[form] if isinstance(form, str) else int(form)
    check(lib().gp_eval_tree_1d(tp, cp, op, len(off) - 1, dptr(X), n_feat or F, N, dptr(y),
                                kind_id(kind), fid, dptr(out), stream_ptr(stream)))


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

    @classmethod
    def boolean(cls, tok, off, n_feat, stream=None):
        """Boolean trees (gp_progset_bool); eval then takes uint32 words and n_cases in bits."""
        tok, tp = _np(tok, np.int32)
        off, op = _np(off, np.int64)
        h = C.c_void_p()
        check(lib().gp_progset_bool(tp, op, len(off) - 1, n_feat, stream_ptr(stream), C.byref(h)))
        return cls(h)

    def eval(self, X, y, kind, out, stream=None, n_cases=None):
        """n_cases: defaults to X.shape[1]; a Boolean set needs the bit count."""
        n = int(X.shape[1]) if n_cases is None else int(n_cases)
        check(lib().gp_progset_eval(self._h, dptr(X), int(X.shape[0]), n, dptr(y),
                                    kind_id(kind), dptr(out), stream_ptr(stream)))

    def eval_noalloc(self, X, y, kind, out, stream=None, n_cases=None):
        """gp_progset_eval_noalloc: the same evaluation with nothing allocated."""
        n = int(X.shape[1]) if n_cases is None else int(n_cases)
        check(lib().gp_progset_eval_noalloc(self._h, dptr(X), int(X.shape[0]), n, dptr(y),
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


# ---------------------------------------------------------------------------
# Batched evaluation and serving
# ---------------------------------------------------------------------------
class Dataset(C.Structure):
    _fields_ = [("X", C.c_void_p), ("n_feat", C.c_int32), ("n_cases", C.c_int64), ("y", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("form", C.c_int32), ("n_prog", C.c_int32), ("dataset", C.c_int32), ("kind", C.c_int32),
                ("tok", C.c_void_p), ("tcst", C.c_void_p), ("toff", C.c_void_p),
                ("code", C.c_void_p), ("loff", C.c_void_p), ("lcst", C.c_void_p), ("lcst_off", C.c_void_p),
                ("n_reg", C.c_int32), ("out", C.c_void_p)]


class BatchConfig(C.Structure):
    _fields_ = [("variant", C.c_int32), ("unit_programs", C.c_int32), ("persistent", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return {"variant": self.variant, "unit_programs": self.unit_programs, "persistent": self.persistent}


class ServeConfig(C.Structure):
    _fields_ = [("memory_budget", C.c_size_t), ("max_queue", C.c_int32), ("n_streams", C.c_int32),
                ("max_batch", C.c_int32), ("batching", C.c_int32), ("dry_run", C.c_int32),
                ("hip_streams", C.c_int32), ("dry_run_gpops", C.c_double)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("cancelled", C.c_int64), ("failed", C.c_int64),
                ("queue_depth", C.c_int32), ("in_flight_batches", C.c_int32), ("bytes_in_flight", C.c_int64),
                ("batches", C.c_int64), ("mean_batch", C.c_double), ("p50_us", C.c_double),
                ("p99_us", C.c_double), ("gpops_per_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def make_job(pop, dataset, kind, out):
    """A gp_job for a synth.TreePop / synth.LinearPop (host arrays are kept
    alive on the returned object)."""
    j = Job()
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    j.n_prog = pop.n_prog
    j.dataset = dataset
    j.kind = kind_id(kind)
    if hasattr(pop, "tok"):
        j.form = 0
        j.tok, j.tcst, j.toff = arr(pop.tok, np.int32), arr(pop.cst, np.float32), arr(pop.off, np.int64)
    else:
        j.form = 1
        j.code, j.loff = arr(pop.code, np.uint32), arr(pop.off, np.int64)
        j.lcst, j.lcst_off = arr(pop.cst, np.float32), arr(pop.cst_off, np.int64)
        j.n_reg = pop.n_reg
    j.out = dptr(out).value if out is not None else None
    j._keep = keep
    return j


def _datasets(ds):
    arr = (Dataset * len(ds))()
    for i, (X, y) in enumerate(ds):
        arr[i].X = X.data_ptr()
        arr[i].n_feat = int(X.shape[0])
        arr[i].n_cases = int(X.shape[1])
        arr[i].y = y.data_ptr() if y is not None else None
    return arr


def gp_eval_batch(datasets, jobs, config=None, stream=None):
    """datasets: list of (X, y) device tensors; jobs: list of Job (make_job)."""
    ds = _datasets(datasets)
    ja = (Job * len(jobs))(*jobs)
    cfg = C.byref(config) if config is not None else None
    check(lib().gp_eval_batch(ds, len(datasets), ja, len(jobs), cfg, stream_ptr(stream)))


def gp_tune_batch(datasets, jobs, reps=3, stream=None):
    ds = _datasets(datasets)
    ja = (Job * len(jobs))(*jobs)
    best = BatchConfig()
    ms = C.c_double()
    check(lib().gp_tune_batch(ds, len(datasets), ja, len(jobs), reps, C.byref(best), C.byref(ms),
                              stream_ptr(stream)))
    return best, ms.value


def variants():
    L = lib()
    out = []
    for i in range(L.gp_num_variants()):
        t, d, f, v, fl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(L.gp_variant_info(i, C.byref(t), C.byref(d), C.byref(f), C.byref(v), C.byref(fl)))
        arith, boolean, trees = bool(fl.value & 1), bool(fl.value & 2), bool(fl.value & 4)
        suffix = "_b" if boolean else (("_at" if arith else "_t") if trees else ("_a" if arith else ""))
        out.append({"t": t.value, "depth": d.value, "n_feat": f.value, "vgprs": v.value, "no_transc": arith,
                    "boolean": boolean, "trees_only": trees,
                    "kernel": "k_core_%d_%d_%d_%d%s" % (t.value, d.value, f.value, v.value, suffix)})
    return out


class Server:
    """gp_serve_*: continuous-batching evaluation server."""

    def __init__(self, memory_budget=0, max_queue=0, n_streams=0, max_batch=0, batching=True,
                 dry_run=False, dry_run_gpops=0.0, hip_streams=0):
        cfg = ServeConfig(memory_budget, max_queue, n_streams, max_batch, 1 if batching else 0,
                          1 if dry_run else 0, hip_streams, dry_run_gpops)
        self._h = C.c_void_p()
        check(lib().gp_serve_create(C.byref(cfg), C.byref(self._h)))
        self._jobs = {}

    def add_dataset(self, X, y, n_feat=None, n_cases=None):
        i = C.c_int32()
        if isinstance(X, int):
            check(lib().gp_serve_add_dataset(self._h, C.c_void_p(X), n_feat, n_cases, C.c_void_p(y), C.byref(i)))
        else:
            check(lib().gp_serve_add_dataset(self._h, dptr(X), int(X.shape[0]), int(X.shape[1]), dptr(y),
                                             C.byref(i)))
        return i.value

    def submit(self, job):
        t = C.c_uint64()
        check(lib().gp_serve_submit(self._h, C.byref(job), C.byref(t)))
        return t.value

    def try_submit(self, job):
        """Returns (status, ticket) instead of raising."""
        t = C.c_uint64()
        rc = lib().gp_serve_submit(self._h, C.byref(job), C.byref(t))
        return rc, t.value

    def poll(self, ticket):
        d = C.c_int32()
        check(lib().gp_serve_poll(self._h, ticket, C.byref(d)))
        return bool(d.value)

    def wait(self, ticket, timeout_us=-1):
        return lib().gp_serve_wait(self._h, ticket, timeout_us)

    def cancel(self, ticket):
        return lib().gp_serve_cancel(self._h, ticket)

    def release(self, ticket):
        return lib().gp_serve_release(self._h, ticket)

    def stats(self):
        st = ServeStats()
        check(lib().gp_serve_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if self._h:
            check(lib().gp_serve_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def core_lower(pop, n_feat, variant, table_base):
    """Core instruction words (uint32, 4 per instruction) and per-program word
    offsets of a synth.TreePop / synth.LinearPop for a kernel variant whose
    handler table is taken to start at table_base (host only)."""
    L = lib()
    nw = C.c_int64()
    prog_off = np.zeros(pop.n_prog + 1, np.int64)
    if hasattr(pop, "tok"):
        a = [np.ascontiguousarray(pop.tok, np.int32), np.ascontiguousarray(pop.cst, np.float32),
             np.ascontiguousarray(pop.off, np.int64)]
        args = [x.ctypes.data for x in a] + [pop.n_prog, n_feat, variant, table_base]
        check(L.gp_core_lower_tree(*args, None, 0, None, C.byref(nw)))
        words = np.zeros(nw.value, np.uint32)
        check(L.gp_core_lower_tree(*args, words.ctypes.data, len(words), prog_off.ctypes.data, C.byref(nw)))
    else:
        a = [np.ascontiguousarray(pop.code, np.uint32), np.ascontiguousarray(pop.off, np.int64),
             np.ascontiguousarray(pop.cst, np.float32), np.ascontiguousarray(pop.cst_off, np.int64)]
        args = [x.ctypes.data for x in a] + [pop.n_prog, pop.n_reg, n_feat, variant, table_base]
        check(L.gp_core_lower_linear(*args, None, 0, None, C.byref(nw)))
        words = np.zeros(nw.value, np.uint32)
        check(L.gp_core_lower_linear(*args, words.ctypes.data, len(words), prog_off.ctypes.data, C.byref(nw)))
    return words, prog_off


def out_tensor(kind, n_prog, n_cases, device="cuda"):
    import torch
    k = kind_id(kind)
    if k in (GP_FIT_HITS, GP_FIT_CLASS_ERR):
        return torch.empty(n_prog, dtype=torch.int32, device=device)
    if k == GP_OUT_CASES:
        return torch.empty((n_prog, n_cases), dtype=torch.float32, device=device)
    return torch.empty(n_prog, dtype=torch.float32, device=device)


# Sources that decide the evaluation kernel's machine code and launch shape.
KERNEL_SOURCES = ("csrc/gen_core.py", "csrc/core_body.h", "csrc/gp_math.h", "csrc/gp_math_tables.h", "csrc/core_kernels.hip",
                  "csrc/core_kernels.h", "csrc/gp_internal.h", "csrc/core_host.cpp", "csrc/core_host.h",
                  "csrc/runtime.cpp", "build.py")


def kernel_source_digest() -> str:
    """Short SHA-256 over the evaluation kernel's sources: a measurement taken
    with another digest describes a different kernel."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()[:16]
