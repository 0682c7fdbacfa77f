"""Seeded synthetic inputs for GP population evaluation.

This module only draws random programs and random data: it builds prefix
trees, linear register programs, feature-major case matrices, noise and the
labels of a linear model.  It evaluates no GP program; target values that come
from a program are computed by whichever evaluator the caller owns.

Program formats (the public interchange format of the evaluation library):

* Prefix trees: ``tok`` int32, opcode in the low 8 bits and, for a variable,
  the feature index in the high 24 bits; ``cst`` float32 parallel to ``tok``
  (the value of a constant token, 0 elsewhere); ``off`` int64 CSR offsets,
  program ``p`` is ``tok[off[p]:off[p+1]]``.
* Linear register programs: ``code`` uint32 words ``op | dst<<8 | src1<<16 |
  src2<<24``; a source id below ``n_reg`` is a register, ids in
  ``[n_reg, n_reg+n_feat)`` are features, ids in ``[128, 256)`` index the
  program's constant table ``cst[cst_off[p] + id-128]``.

Every generator takes an explicit ``numpy.random.Generator`` (PCG64) so that
the GPU path, the oracle and the benchmark see identical arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Opcodes of the interchange format.
ADD, SUB, MUL, PDIV, SIN, COS, EXPC, PLOG = 0, 1, 2, 3, 4, 5, 6, 7
VAR, CONST = 64, 65
ARITY = {ADD: 2, SUB: 2, MUL: 2, PDIV: 2, SIN: 1, COS: 1, EXPC: 1, PLOG: 1}
NAMES = {ADD: "+", SUB: "-", MUL: "*", PDIV: "/", SIN: "sin", COS: "cos",
         EXPC: "exp", PLOG: "log"}
BASIC = (ADD, SUB, MUL, PDIV)
FULL = (ADD, SUB, MUL, PDIV, SIN, COS, EXPC, PLOG)
ARITH3 = (ADD, SUB, MUL)
# Boolean function set (sub-machine-code GP: 32 bit-packed cases per word)
AND, OR, NAND, NOR = 8, 9, 10, 11
ARITY.update({AND: 2, OR: 2, NAND: 2, NOR: 2})
NAMES.update({AND: "and", OR: "or", NAND: "nand", NOR: "nor"})
BOOL_SET = (AND, OR, NAND, NOR)
# Classification functions (the Shuttle and KDD Cup 99 problems); in arithmetic
# trees AND and OR are the logical functions.  IF is the one three-operand function.
GT, LT, EQ, IF = 12, 13, 14, 15
ARITY.update({GT: 2, LT: 2, EQ: 2, IF: 3})
NAMES.update({GT: ">", LT: "<", EQ: "==", IF: "if"})
SHUTTLE_SET = (MUL, PDIV, ADD, SUB, GT, LT, EQ, AND, OR, IF)
KDD_SET = (ADD, SUB, MUL, PDIV, GT, LT, EQ, AND, OR, IF, SIN, COS, PLOG, EXPC)

SRC_CONST_BASE = 128


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# Program containers
# ----------------------------------------------------------------------------
@dataclass
class TreePop:
    tok: np.ndarray            # int32
    cst: np.ndarray            # float32
    off: np.ndarray            # int64, len P+1

    @property
    def n_prog(self) -> int:
        return len(self.off) - 1

    def sizes(self) -> np.ndarray:
        return np.diff(self.off)

    def program(self, p: int):
        a, b = int(self.off[p]), int(self.off[p + 1])
        return self.tok[a:b], self.cst[a:b]

    def subset(self, idx) -> "TreePop":
        return trees_from_lists([self.program(int(i)) for i in idx])


@dataclass
class LinearPop:
    code: np.ndarray           # uint32
    off: np.ndarray            # int64, len P+1
    cst: np.ndarray            # float32
    cst_off: np.ndarray        # int64, len P+1
    n_reg: int = 8

    @property
    def n_prog(self) -> int:
        return len(self.off) - 1

    def sizes(self) -> np.ndarray:
        return np.diff(self.off)

    def subset(self, idx) -> "LinearPop":
        code, cst = [], []
        for i in idx:
            i = int(i)
            code.append(self.code[self.off[i]:self.off[i + 1]])
            cst.append(self.cst[self.cst_off[i]:self.cst_off[i + 1]])
        return linear_from_lists(code, cst, self.n_reg)


def trees_from_lists(progs) -> TreePop:
    """progs: iterable of (tok, cst) pairs."""
    toks, csts, off = [], [], [0]
    for t, c in progs:
        t = np.asarray(t, dtype=np.int32)
        c = np.asarray(c, dtype=np.float32)
        toks.append(t)
        csts.append(c)
        off.append(off[-1] + len(t))
    tok = np.concatenate(toks) if toks else np.zeros(0, np.int32)
    cst = np.concatenate(csts) if csts else np.zeros(0, np.float32)
    return TreePop(tok.astype(np.int32), cst.astype(np.float32),
                   np.asarray(off, dtype=np.int64))


def linear_from_lists(codes, csts, n_reg: int = 8) -> LinearPop:
    off, coff = [0], [0]
    for c, k in zip(codes, csts):
        off.append(off[-1] + len(c))
        coff.append(coff[-1] + len(k))
    code = np.concatenate([np.asarray(c, np.uint32) for c in codes]) if codes else np.zeros(0, np.uint32)
    cst = np.concatenate([np.asarray(k, np.float32) for k in csts]) if csts else np.zeros(0, np.float32)
    return LinearPop(code.astype(np.uint32), np.asarray(off, np.int64),
                     cst.astype(np.float32), np.asarray(coff, np.int64), n_reg)


def var_tok(k: int) -> int:
    return VAR | (k << 8)


def lin_word(op: int, dst: int, s1: int, s2: int) -> int:
    return (op & 0xFF) | ((dst & 0xFF) << 8) | ((s1 & 0xFF) << 16) | ((s2 & 0xFF) << 24)


# ----------------------------------------------------------------------------
# Tree generators
# ----------------------------------------------------------------------------
def _terminal(rng, n_feat, p_const, crange):
    if rng.random() < p_const:
        return CONST, np.float32(rng.uniform(crange[0], crange[1]))
    return var_tok(int(rng.integers(n_feat))), np.float32(0.0)


def _grow_full(rng, depth, full, fset, n_feat, p_const, crange, out_t, out_c):
    # Prefix emission.  Depth 0 means "a terminal here".
    n_fun = len(fset)
    if depth == 0:
        t, c = _terminal(rng, n_feat, p_const, crange)
        out_t.append(t); out_c.append(c)
        return
    if not full:
        # grow: any primitive, terminals weighted by the size of the terminal set
        n_term = n_feat + (1 if p_const > 0 else 0)
        if rng.random() < n_term / (n_term + n_fun):
            t, c = _terminal(rng, n_feat, p_const, crange)
            out_t.append(t); out_c.append(c)
            return
    f = fset[int(rng.integers(n_fun))]
    out_t.append(f); out_c.append(np.float32(0.0))
    for _ in range(ARITY[f]):
        _grow_full(rng, depth - 1, full, fset, n_feat, p_const, crange, out_t, out_c)


def random_tree(rng, depth, full, fset, n_feat, p_const, crange=(-1.0, 1.0)):
    t, c = [], []
    _grow_full(rng, depth, full, fset, n_feat, p_const, crange, t, c)
    return np.asarray(t, np.int32), np.asarray(c, np.float32)


def ramped_half_and_half(rng, n, fset, n_feat, dmin, dmax, max_nodes,
                         p_const=0.5, crange=(-1.0, 1.0)) -> TreePop:
    """Koza's ramped half-and-half: depths cycle over [dmin, dmax], alternate
    grow and full; trees larger than max_nodes are re-drawn."""
    progs = []
    depths = list(range(dmin, dmax + 1))
    i = 0
    while len(progs) < n:
        d = depths[(i // 2) % len(depths)]
        full = (i % 2) == 1
        i += 1
        t, c = random_tree(rng, d, full, fset, n_feat, p_const, crange)
        if len(t) > max_nodes:
            continue
        progs.append((t, c))
    return trees_from_lists(progs)


def ptc2_tree(rng, target, fset, n_feat, p_const, crange=(-1.0, 1.0)):
    """Luke's PTC2 size-targeted growth: expand randomly chosen open argument
    slots with functions until the node count plus the open slots reaches the
    target, then close every open slot with a terminal.  Returns prefix arrays
    with at most ``target`` nodes (a single terminal when target == 1)."""
    if target <= 1:
        t, c = _terminal(rng, n_feat, p_const, crange)
        return np.asarray([t], np.int32), np.asarray([c], np.float32)
    # node records: (op, children list)
    ops = []
    kids = []
    open_slots = []           # (parent, position)
    def new_fun(f):
        ops.append(f)
        kids.append([-1] * ARITY[f])
        idx = len(ops) - 1
        for pos in range(ARITY[f]):
            open_slots.append((idx, pos))
        return idx

    roots = [g for g in fset if 1 + ARITY[g] <= target]
    if not roots:
        t, c = _terminal(rng, n_feat, p_const, crange)
        return np.asarray([t], np.int32), np.asarray([c], np.float32)
    new_fun(roots[int(rng.integers(len(roots)))])
    n_nodes = 1
    while open_slots:
        # a function added at an open slot grows the final size by its arity
        choices = [g for g in fset if n_nodes + len(open_slots) + ARITY[g] - 1 + 1 <= target]
        if n_nodes + len(open_slots) >= target or not choices:
            break
        j = int(rng.integers(len(open_slots)))
        parent, pos = open_slots[j]
        open_slots[j] = open_slots[-1]
        open_slots.pop()
        g = choices[int(rng.integers(len(choices)))]
        child = new_fun(g)
        kids[parent][pos] = child
        n_nodes += 1
    for parent, pos in open_slots:
        t, c = _terminal(rng, n_feat, p_const, crange)
        ops.append(("T", t, c))
        kids.append([])
        kids[parent][pos] = len(ops) - 1
    # prefix emission (iterative)
    out_t, out_c = [], []
    stack = [0]
    while stack:
        i = stack.pop()
        o = ops[i]
        if isinstance(o, tuple):
            out_t.append(o[1]); out_c.append(o[2])
        else:
            out_t.append(o); out_c.append(np.float32(0.0))
            for ch in reversed(kids[i]):
                stack.append(ch)
    return np.asarray(out_t, np.int32), np.asarray(out_c, np.float32)


def ptc2_population(rng, n, fset, n_feat, size_lo, size_hi, p_const,
                    crange=(-1.0, 1.0), sizes=None) -> TreePop:
    progs = []
    for i in range(n):
        target = int(sizes[i]) if sizes is not None else int(rng.integers(size_lo, size_hi + 1))
        progs.append(ptc2_tree(rng, target, fset, n_feat, p_const, crange))
    return trees_from_lists(progs)


# ----------------------------------------------------------------------------
# Linear register programs
# ----------------------------------------------------------------------------
def linear_population(rng, n, len_lo, len_hi, ops, n_reg, n_feat, n_const=0,
                      crange=(-1.0, 1.0), lengths=None) -> LinearPop:
    """dst uniform over registers; sources uniform over registers, features
    and (if n_const > 0) the program's constants."""
    codes, csts = [], []
    n_src = n_reg + n_feat + n_const
    ops = np.asarray(ops, np.uint32)
    for i in range(n):
        L = int(lengths[i]) if lengths is not None else int(rng.integers(len_lo, len_hi + 1))
        op = ops[rng.integers(len(ops), size=L)]
        dst = rng.integers(n_reg, size=L).astype(np.uint32)
        s = rng.integers(n_src, size=(2, L)).astype(np.uint32)
        s = np.where(s >= n_reg + n_feat, s - (n_reg + n_feat) + SRC_CONST_BASE, s)
        code = op | (dst << 8) | (s[0] << 16) | (s[1] << 24)
        codes.append(code.astype(np.uint32))
        csts.append(rng.uniform(crange[0], crange[1], size=n_const).astype(np.float32))
    return linear_from_lists(codes, csts, n_reg)


# ----------------------------------------------------------------------------
# Case matrices and targets
# ----------------------------------------------------------------------------
def uniform_cases(rng, n_feat, n_cases, lo, hi) -> np.ndarray:
    """Feature-major float32 matrix X[f, c]."""
    return rng.uniform(lo, hi, size=(n_feat, n_cases)).astype(np.float32)


def normal_cases(rng, n_feat, n_cases) -> np.ndarray:
    return rng.standard_normal(size=(n_feat, n_cases)).astype(np.float32)


def gaussian_noise(rng, n_cases, sigma) -> np.ndarray:
    return (rng.standard_normal(n_cases) * sigma).astype(np.float32)


def sign_labels(rng, X: np.ndarray):
    """Labels of a random linear model: w ~ N(0,1)^F; s = w0*x0 + w1*x1 + ...
    accumulated left to right in float32 (each product and each sum rounded
    to binary32); label +1 where s > 0, else -1.  Returns (w, y)."""
    F = X.shape[0]
    w = rng.standard_normal(F).astype(np.float32)
    s = np.zeros(X.shape[1], np.float32)
    for f in range(F):
        s = (s + (w[f] * X[f]).astype(np.float32)).astype(np.float32)
    y = np.where(s > np.float32(0.0), np.float32(1.0), np.float32(-1.0)).astype(np.float32)
    return w, y


def lognormal_lengths(rng, n, mu, sigma, lo, hi) -> np.ndarray:
    v = np.rint(rng.lognormal(mu, sigma, size=n))
    return np.clip(v, lo, hi).astype(np.int64)


# ----------------------------------------------------------------------------
# Workloads (the paper-shaped synthetic configurations)
# ----------------------------------------------------------------------------
@dataclass
class TreeWorkload:
    name: str
    pop: TreePop
    X: np.ndarray              # (F, N) float32
    target: TreePop            # candidate target trees, first acceptable one is used
    noise: np.ndarray          # (N,) float32 added to the target values
    kind: str                  # "sum_abs" | "mse" | "hits"
    fset: tuple
    meta: dict = field(default_factory=dict)


@dataclass
class LinearWorkload:
    name: str
    pop: LinearPop
    X: np.ndarray
    y: np.ndarray
    kind: str
    meta: dict = field(default_factory=dict)


def tiny_tree_workload(seed: int = 1, n_prog: int = 100, n_cases: int = 1024) -> TreeWorkload:
    """100 ramped half-and-half trees (depth 2-6, <=64 nodes) over {+,-,*,/p},
    terminals {x0, U(-1,1) constant} with probability 1/2 each; 1024 cases
    x0 ~ U(-1,1); target values from one full depth-5 tree; sum |error|."""
    rng = rng_for(seed)
    pop = ramped_half_and_half(rng, n_prog, BASIC, 1, 2, 6, 64, p_const=0.5)
    X = uniform_cases(rng, 1, n_cases, -1.0, 1.0)
    tt, tc = random_tree(rng, 5, True, BASIC, 1, 0.5)
    target = trees_from_lists([(tt, tc)])
    return TreeWorkload("tiny-tree-100x1024", pop, X, target,
                        np.zeros(n_cases, np.float32), "sum_abs", BASIC,
                        dict(n_feat=1, n_cases=n_cases, n_prog=n_prog))


def scale_tree_workload(seed: int = 2, n_prog: int = 4096, n_cases: int = 65536,
                        n_feat: int = 8, fset=FULL, max_size: int = 256,
                        n_target_candidates: int = 16) -> TreeWorkload:
    """4096 PTC2 trees of size U{1..256} over the given function set,
    terminals x0..x7 and a U(-1,1) constant drawn uniformly among the nine;
    cases X ~ U(-5,5) feature-major; target = first candidate tree whose
    values are all finite with |y| < 1e6, plus N(0, sigma=0.01) noise; MSE."""
    rng = rng_for(seed)
    p_const = 1.0 / (n_feat + 1)
    pop = ptc2_population(rng, n_prog, fset, n_feat, 1, max_size, p_const)
    X = uniform_cases(rng, n_feat, n_cases, -5.0, 5.0)
    cands = [ptc2_tree(rng, int(rng.integers(8, 33)), fset, n_feat, p_const)
             for _ in range(n_target_candidates)]
    target = trees_from_lists(cands)
    noise = gaussian_noise(rng, n_cases, 0.01)
    name = "scale-tree-%dx%d-F%d-%s" % (n_prog, n_cases, n_feat,
                                        "full" if tuple(fset) == FULL else "arith")
    return TreeWorkload(name, pop, X, target, noise, "mse", tuple(fset),
                        dict(n_feat=n_feat, n_cases=n_cases, n_prog=n_prog))


def linear_workload(seed: int = 3, n_prog: int = 4096, n_cases: int = 1 << 20,
                    n_reg: int = 8, n_feat: int = 16, len_lo: int = 32,
                    len_hi: int = 256) -> LinearWorkload:
    """4096 register programs of U{32..256} instructions over {+,-,*,/p},
    dst uniform over 8 registers, sources uniform over the 24 register and
    feature ids, no constants; X ~ N(0,1); labels = sign of a random linear
    model; fitness = hit count."""
    rng = rng_for(seed)
    pop = linear_population(rng, n_prog, len_lo, len_hi, BASIC, n_reg, n_feat)
    X = normal_cases(rng, n_feat, n_cases)
    w, y = sign_labels(rng, X)
    return LinearWorkload("linear-%dx%d-R%d-F%d" % (n_prog, n_cases, n_reg, n_feat),
                          pop, X, y, "hits", dict(w=w, n_feat=n_feat, n_cases=n_cases))


def wl_scaled_tree(seed, n_prog, n_cases, n_feat=8, fset=FULL, max_size=256):
    return scale_tree_workload(seed, n_prog, n_cases, n_feat, fset, max_size)


# ----------------------------------------------------------------------------
# Batched and served workloads
# ----------------------------------------------------------------------------
@dataclass
class BatchJobSpec:
    pop: object                # TreePop or LinearPop
    dataset: int
    kind: str


@dataclass
class BatchedWorkload:
    name: str
    X: list                    # per dataset, (F, N) float32
    target: list               # per dataset, TreePop of candidate target trees
    noise: list                # per dataset, (N,) float32
    jobs: list                 # BatchJobSpec
    meta: dict = field(default_factory=dict)


def batched_workload(seed: int = 4, n_prog: int = 10000, n_jobs: int = 40,
                     sizes=(4096, 65536, 1 << 20), n_feat: int = 8) -> BatchedWorkload:
    """Several GP populations over three resident case matrices, evaluated in
    one launch: 10,000 programs split into 40 populations of 250, even ones
    PTC2 trees over the full function set, odd ones register programs over
    {+,-,*,/p} with 8 registers and 2 constants; program lengths
    round(lognormal(ln 64, 1)) clipped to [8, 1024]; each population's case
    matrix drawn uniformly from the three (4096 / 65,536 / 1,048,576 cases x
    8 features ~U(-5,5)); targets from a random tree plus N(0, 0.01) noise;
    fitness = MSE."""
    rng = rng_for(seed)
    X, target, noise = [], [], []
    p_const = 1.0 / (n_feat + 1)
    for n in sizes:
        X.append(uniform_cases(rng, n_feat, n, -5.0, 5.0))
        target.append(trees_from_lists([ptc2_tree(rng, int(rng.integers(8, 33)), FULL, n_feat, p_const)
                                        for _ in range(16)]))
        noise.append(gaussian_noise(rng, n, 0.01))
    per = n_prog // n_jobs
    jobs = []
    for j in range(n_jobs):
        lens = lognormal_lengths(rng, per, math.log(64.0), 1.0, 8, 1024)
        ds = int(rng.integers(len(sizes)))
        if j % 2 == 0:
            pop = ptc2_population(rng, per, FULL, n_feat, 0, 0, p_const, sizes=lens)
        else:
            pop = linear_population(rng, per, 0, 0, BASIC, 8, n_feat, n_const=2, lengths=lens)
        jobs.append(BatchJobSpec(pop, ds, "mse"))
    return BatchedWorkload("batched-%dprogs-%djobs-N%s-F%d" % (n_prog, n_jobs, "/".join(str(s) for s in sizes), n_feat),
                           X, target, noise, jobs,
                           dict(n_prog=n_prog, n_jobs=n_jobs, sizes=list(sizes), n_feat=n_feat))


@dataclass
class ServedRun:
    X: np.ndarray              # (F, N) float32
    target: TreePop            # candidate target trees
    noise: np.ndarray
    requests: list             # per request: (form, start, n_prog) into the program pools
    think_s: np.ndarray        # think time after each request, seconds


@dataclass
class ServedWorkload:
    name: str
    runs: list                 # ServedRun
    tree_pool: TreePop         # programs over MAX_SERVE_FEAT features
    lin_pool: LinearPop
    meta: dict = field(default_factory=dict)


MAX_SERVE_FEAT = 32


def served_workload(seed: int = 5, n_runs: int = 32, n_req: int = 16, pool: int = 8192,
                    n_lo: int = 1000, n_hi: int = 2_000_000, pop_lo: int = 64, pop_hi: int = 8192,
                    len_hi: int = 512, think_mean_s: float = 0.002) -> ServedWorkload:
    """Concurrent GP runs, each with its own resident case matrix: cases
    log-uniform in [1k, 2M], features uniform in {4..32}, X ~U(-5,5), targets
    from a random tree plus N(0, 0.01) noise, MSE.  Each run issues n_req
    population evaluations in a closed loop (submit, wait for the result,
    think for an Exp(2 ms) time): population log-uniform in [64, 8192],
    program lengths U{1..512}, tree or register form with probability 1/2.
    Programs are slices of two shared pools drawn over 32 features; a request
    to a run with F features reads feature k as k mod F (remap_features)."""
    rng = rng_for(seed)
    p_const = 1.0 / (MAX_SERVE_FEAT + 1)
    tree_pool = ptc2_population(rng, pool, FULL, MAX_SERVE_FEAT, 1, len_hi, p_const)
    lin_pool = linear_population(rng, pool, 1, len_hi, BASIC, 8, MAX_SERVE_FEAT, n_const=2)
    runs = []
    for r in range(n_runs):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        F = int(rng.integers(4, MAX_SERVE_FEAT + 1))
        X = uniform_cases(rng, F, N, -5.0, 5.0)
        tgt = trees_from_lists([ptc2_tree(rng, int(rng.integers(8, 33)), FULL, F, 1.0 / (F + 1))
                                for _ in range(16)])
        noise = gaussian_noise(rng, N, 0.01)
        reqs = []
        for _ in range(n_req):
            P = int(round(math.exp(rng.uniform(math.log(pop_lo), math.log(pop_hi)))))
            form = int(rng.integers(2))
            start = int(rng.integers(pool))
            reqs.append((form, start, P))
        think = rng.exponential(think_mean_s, size=n_req)
        runs.append(ServedRun(X, tgt, noise, reqs, think))
    return ServedWorkload("served-%druns-%dreq" % (n_runs, n_req), runs, tree_pool, lin_pool,
                          dict(n_runs=n_runs, n_req=n_req, pool=pool))


def pool_slice(pool, start: int, n: int):
    """Programs start, start+1, ... (wrapping) of a TreePop / LinearPop."""
    P = pool.n_prog
    if n > P:
        raise ValueError("slice longer than the pool")
    pieces = [(start, min(P, start + n))]
    if start + n > P:
        pieces.append((0, start + n - P))
    if hasattr(pool, "tok"):
        tok, cst, off = [], [], [np.zeros(1, np.int64)]
        base = 0
        for a, b in pieces:
            lo, hi = int(pool.off[a]), int(pool.off[b])
            tok.append(pool.tok[lo:hi])
            cst.append(pool.cst[lo:hi])
            off.append(pool.off[a + 1:b + 1] - lo + base)
            base += hi - lo
        return TreePop(np.concatenate(tok), np.concatenate(cst), np.concatenate(off))
    code, off, cst, coff = [], [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)]
    base = cbase = 0
    for a, b in pieces:
        lo, hi = int(pool.off[a]), int(pool.off[b])
        clo, chi = int(pool.cst_off[a]), int(pool.cst_off[b])
        code.append(pool.code[lo:hi])
        cst.append(pool.cst[clo:chi])
        off.append(pool.off[a + 1:b + 1] - lo + base)
        coff.append(pool.cst_off[a + 1:b + 1] - clo + cbase)
        base += hi - lo
        cbase += chi - clo
    return LinearPop(np.concatenate(code), np.concatenate(off), np.concatenate(cst), np.concatenate(coff),
                     pool.n_reg)


def remap_features(pop, n_feat: int):
    """The same programs reading feature k mod n_feat instead of feature k."""
    if hasattr(pop, "tok"):
        tok = pop.tok.copy()
        v = (tok & 0xFF) == VAR
        k = tok >> 8
        tok[v] = VAR | ((k[v] % n_feat) << 8)
        return TreePop(tok, pop.cst, pop.off)
    code = pop.code.copy()
    R = pop.n_reg
    out = code
    for sh in (16, 24):
        s = (code >> sh) & 0xFF
        feat = (s >= R) & (s < SRC_CONST_BASE)
        s2 = np.where(feat, R + (s - R) % n_feat, s)
        out = (out & ~np.uint32(0xFF << sh)) | (s2.astype(np.uint32) << sh)
    return LinearPop(out.astype(np.uint32), pop.off, pop.cst, pop.cst_off, pop.n_reg)


# ----------------------------------------------------------------------------
# Boolean multiplexer (bit-packed, exhaustive)
# ----------------------------------------------------------------------------
def pack_bits(bits) -> np.ndarray:
    """Pack a 0/1 array of cases into uint32 words: bit b of word w is case
    32 w + b (the last word zero-padded)."""
    bits = np.asarray(bits, np.uint8)
    pad = (-len(bits)) % 32
    if pad:
        bits = np.concatenate([bits, np.zeros(pad, np.uint8)])
    return np.packbits(bits, bitorder="little").view("<u4").astype(np.uint32)


def mux_cases(k: int):
    """All cases of the k-address multiplexer (k + 2^k inputs): input f of
    case c is bit f of c; inputs 0 .. k-1 are the address bits A0 (least
    significant) .. A(k-1), input k + d is data bit Dd; the target is the
    data bit the address selects.  Returns (Xw (n_in, W) uint32, yw (W,)
    uint32, n_cases)."""
    n_in = k + (1 << k)
    n_cases = 1 << n_in
    c = np.arange(n_cases, dtype=np.uint64)
    Xw = np.stack([pack_bits((c >> np.uint64(f)) & np.uint64(1)) for f in range(n_in)])
    addr = c & np.uint64((1 << k) - 1)
    y = (c >> (np.uint64(k) + addr)) & np.uint64(1)
    return Xw, pack_bits(y), n_cases


@dataclass
class BoolWorkload:
    name: str
    pop: TreePop
    Xw: np.ndarray             # (F, W) uint32
    yw: np.ndarray             # (W,) uint32
    n_cases: int
    meta: dict = field(default_factory=dict)


def mux_workload(seed: int = 6, k: int = 4, n_prog: int = 4096, max_size: int = 256) -> BoolWorkload:
    """The 20-multiplexer (k = 4: A0-A3, D0-D15) over all 2^20 cases,
    bit-packed into 32,768 words per input; 4096 PTC2 trees of size
    U{1..256} over {AND, OR, NAND, NOR} with the 20 inputs as terminals;
    fitness = number of correctly classified cases."""
    rng = rng_for(seed)
    Xw, yw, n_cases = mux_cases(k)
    pop = ptc2_population(rng, n_prog, BOOL_SET, Xw.shape[0], 1, max_size, 0.0)
    return BoolWorkload("mux%d-%dx%d" % (Xw.shape[0], n_prog, n_cases), pop, Xw, yw, n_cases,
                        dict(k=k, n_in=Xw.shape[0]))


# ----------------------------------------------------------------------------
# Classification (stand-ins shaped like the Shuttle and KDD Cup 99 problems)
# ----------------------------------------------------------------------------
@dataclass
class ClassWorkload:
    name: str
    pop: TreePop
    X: np.ndarray              # (F, N) float32
    y: np.ndarray              # (N,) float32 class indices
    n_classes: int
    kind: str = "class_err"
    meta: dict = field(default_factory=dict)


def class_labels(rng, n_cases, probs) -> np.ndarray:
    """Class indices drawn with the given class probabilities."""
    p = np.asarray(probs, np.float64)
    return rng.choice(len(p), size=n_cases, p=p / p.sum()).astype(np.int64)


def _tail_probs(head, n_classes):
    """The head probabilities, then the rest of the mass over the remaining
    classes halving from one class to the next."""
    rest = n_classes - len(head)
    w = 0.5 ** np.arange(rest)
    return list(head) + list((1.0 - sum(head)) * w / w.sum())


def shuttle_cases(rng, n_cases=58000, n_feat=9, n_classes=10):
    """Shuttle-shaped cases: 9 integer-valued inputs, 10 classes with 75 % of
    the cases in one of them; each class has its own centre in [-100, 100]
    per input and the inputs scatter around it with sigma 15."""
    y = class_labels(rng, n_cases, _tail_probs([0.75], n_classes))
    centre = rng.uniform(-100.0, 100.0, size=(n_classes, n_feat))
    X = np.rint(centre[y].T + rng.normal(0.0, 15.0, size=(n_feat, n_cases))).astype(np.float32)
    return np.ascontiguousarray(X), y.astype(np.float32)


def kdd_cases(rng, n_cases=494021, n_feat=41, n_classes=22):
    """KDD-Cup-99-shaped cases: 41 inputs, 22 classes, three of them holding
    57 %, 22 % and 20 % of the cases.  Inputs come in four kinds by index mod
    4: counts in 0..511, rates in [0, 1] with two decimals, heavy-tailed
    byte counts (lognormal, up to about 1e7) and small integers in 0..10;
    each class shifts every input's distribution its own way."""
    y = class_labels(rng, n_cases, _tail_probs([0.568, 0.217, 0.197], n_classes))
    shift = rng.uniform(0.0, 1.0, size=(n_classes, n_feat))
    X = np.empty((n_feat, n_cases), np.float32)
    for f in range(n_feat):
        s = shift[y, f]
        k = f % 4
        if k == 0:
            v = np.minimum(511, rng.poisson(1.0 + 300.0 * s))
        elif k == 1:
            v = np.round(np.clip(s + rng.normal(0.0, 0.1, n_cases), 0.0, 1.0), 2)
        elif k == 2:
            v = np.round(np.minimum(1e7, rng.lognormal(2.0 + 8.0 * s, 1.5)))
        else:
            v = np.minimum(10, rng.poisson(0.2 + 5.0 * s))
        X[f] = v
    return X, y.astype(np.float32)


def shuttle_workload(seed: int = 7, n_prog: int = 4096, n_cases: int = 58000, max_size: int = 256) -> ClassWorkload:
    """The Shuttle problem's shape: 58,000 cases x 9 inputs, 10 classes;
    4096 PTC2 trees of size U{1..256} over {*, /, +, -, >, <, ==, AND, OR,
    IF} with the 9 inputs and constants U(-200, 200) as terminals (a
    constant with probability 1/10); fitness = incorrect classifications."""
    rng = rng_for(seed)
    X, y = shuttle_cases(rng, n_cases)
    F = X.shape[0]
    pop = ptc2_population(rng, n_prog, SHUTTLE_SET, F, 1, max_size, 1.0 / (F + 1), crange=(-200.0, 200.0))
    return ClassWorkload("shuttle-%dx%d-F%d-C10" % (n_prog, n_cases, F), pop, X, y, 10,
                         meta=dict(n_feat=F, n_classes=10))


def kdd_workload(seed: int = 8, n_prog: int = 4096, n_cases: int = 494021, max_size: int = 256) -> ClassWorkload:
    """The KDD Cup 99 problem's shape: 494,021 cases x 41 inputs, 22 classes;
    4096 PTC2 trees of size U{1..256} over {+, -, *, /, >, <, ==, AND, OR,
    IF, sin, cos, log, exp} with the 41 inputs and constants U(-20000,
    20000) as terminals (a constant with probability 1/42); fitness =
    incorrect classifications."""
    rng = rng_for(seed)
    X, y = kdd_cases(rng, n_cases)
    F = X.shape[0]
    pop = ptc2_population(rng, n_prog, KDD_SET, F, 1, max_size, 1.0 / (F + 1), crange=(-20000.0, 20000.0))
    return ClassWorkload("kdd-%dx%d-F%d-C22" % (n_prog, n_cases, F), pop, X, y, 22,
                         meta=dict(n_feat=F, n_classes=22))
