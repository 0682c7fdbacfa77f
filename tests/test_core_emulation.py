"""The hand-written interpreter core, executed on the CPU.

The generated handler code (the same instruction text the kernel assembles)
is run by a small emulator of the instructions it uses: scalar moves, adds
and shifts, the scalar load of the next instruction, the jump to its
handler's address, the VGPR index mode and the FP32 vector operations.
Programs are translated by the library (gp_core_lower_*), with the handler
table placed at a chosen address; the work the kernel does outside the core
(feature loading, protected division and transcendental exits, reading the
result) is mirrored here.  Outputs must equal the oracle's bit for bit.

This checks the slot arithmetic, every handler's operand offsets and the
host translation before any of it runs on a GPU."""
import math
import os
import re
import sys

import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth

CSRC = os.path.join(os.path.dirname(gp.__file__), "csrc")
sys.path.insert(0, CSRC)
import gen_core  # noqa: E402

sys.path.pop(0)

BASE = 0x7F12345600C0 & ~63


def f32(x):
    return np.float32(x)


class CoreEmu:
    def __init__(self, variant_index):
        T, D, NF, NCV, mode = gen_core.VARIANTS[variant_index]
        tag, V0, FO, hs, nslots = gen_core.gen_variant(T, D, NF, NCV, mode)
        self.T, self.D, self.NF, self.V0, self.FO = T, D, NF, V0, FO
        self.by_slot = {h.slot: h for h in hs}
        self.prog = {h.slot: [self._parse(x) for x in h.lines] for h in hs}
        self.v = np.zeros((256, 64), np.float32)
        self.s = [0] * 128
        self.vcc = np.zeros(64, bool)
        self.smask = np.zeros(64, bool)
        self.steps = 0

    # ------------------------------------------------------------------ parse
    @staticmethod
    def _reg(tok):
        tok = tok.strip()
        if tok == "vcc":
            return ("vcc", 0)
        if tok.startswith("s["):
            return ("sp", int(tok[2:].split(":")[0]))
        if tok.startswith("-v"):
            return ("vneg", int(tok[2:]))
        if tok.startswith("|v"):
            return ("vabs", int(tok[2:-1]))
        if tok.startswith("v"):
            return ("v", int(tok[1:]))
        if tok.startswith("s"):
            return ("s", int(tok[1:]))
        if "." in tok:
            return ("f", float(tok))
        return ("i", int(tok, 0))

    def _parse(self, line):
        m = re.match(r"(\S+)\s*(.*)", line)
        op, rest = m.group(1), m.group(2)
        if op == "s_set_gpr_idx_on":
            r, modes = re.match(r"(s\d+), gpr_idx\(([A-Z0-9,]*)\)", rest).groups()
            return (op, int(r[1:]), set(modes.split(",")))
        if op in ("s_set_gpr_idx_off", "s_waitcnt", "s_nop"):
            return (op,)
        if op == "s_load_dwordx8":
            assert rest == "s[64:71], s[60:61], s62", rest
            return (op,)
        if op == "s_setpc_b64":
            assert rest in ("s[64:65]", "s[68:69]"), rest
            return (op, int(rest[2:4]))
        if op == "s_branch":
            assert ".Lgpx_end_" in rest
            return (op,)
        if op == "v_bitop3_b32":
            regs, table = rest.split(" bitop3:")
            return (op, [self._reg(a) for a in regs.split(",")] + [("t", int(table, 0))])
        args = [self._reg(a) for a in rest.split(",")]
        return (op, args)

    # ------------------------------------------------------------------ run
    def run(self, code, off):
        """Run from byte offset `off` until the exit handler; returns
        (offset, payload, constant) as the asm block hands them back."""
        s = self.s
        s[62] = off
        # entry: this record and the next one, then the phase-A handler
        for k in range(8):
            s[64 + k] = int(code[off // 4 + k])
        idx_on, m0, modes = False, 0, set()
        pair = 64
        while True:
            addr = s[pair] | (s[pair + 1] << 32)
            rel = addr - BASE
            assert rel >= 0 and rel % gen_core.SLOT == 0, hex(addr)
            slot = rel // gen_core.SLOT
            assert slot in self.prog, slot
            for ins in self.prog[slot]:
                self.steps += 1
                op = ins[0]
                if op == "s_set_gpr_idx_on":
                    idx_on, m0, modes = True, s[ins[1]] & 255, ins[2]
                elif op == "s_set_gpr_idx_off":
                    idx_on = False
                elif op in ("s_waitcnt", "s_nop"):
                    pass
                elif op == "s_load_dwordx8":
                    o = s[62] // 4
                    for k in range(8):
                        s[64 + k] = int(code[o + k])
                elif op == "s_setpc_b64":
                    pair = ins[1]
                    break
                elif op == "s_branch":
                    return s[62], s[66], s[67]
                elif op == "s_mov_b32":
                    (_, d), (k, a) = ins[1]
                    s[d] = s[a] if k == "s" else a
                elif op == "s_add_u32":
                    (_, d), (_, a), (_, b) = ins[1]
                    s[d] = (s[a] + b) & 0xFFFFFFFF
                elif op == "s_lshr_b32":
                    (_, d), (_, a), (_, b) = ins[1]
                    s[d] = s[a] >> b
                elif op in ("s_and_b64", "s_or_b64"):
                    assert [a[0] for a in ins[1]] == ["vcc", "vcc", "sp"], ins
                    self.vcc = (self.vcc & self.smask) if op == "s_and_b64" else (self.vcc | self.smask)
                else:
                    self._valu(op, ins[1], idx_on, m0, modes)
            else:
                raise AssertionError("handler fell through")

    def _valu(self, op, args, idx_on, m0, modes):
        def src(k, a, field):
            if k == "s":
                return np.full(64, np.frombuffer(np.uint32(self.s[a]).tobytes(), np.float32)[0])
            if k in ("f", "i"):
                return np.full(64, np.float32(a))
            r = a + (m0 if idx_on and field in modes else 0)
            assert 0 <= r < 256
            if k == "vneg":
                return -self.v[r]
            if k == "vabs":
                return np.abs(self.v[r])
            return self.v[r]
        if args[0][0] in ("vcc", "sp"):   # a compare: its destination is a mask register
            self._div_op(op, args, args[0][0], src)
            return
        (_, d) = args[0]
        dr = d + (m0 if idx_on and "DST" in modes else 0)
        # the core's range, or the division handlers' temporaries below it
        assert self.V0 - gen_core.DIV_TMP <= dr < 256, dr
        if dr < self.V0:
            assert not (idx_on and "DST" in modes)
        if op == "v_mov_b32_e32":
            self.v[dr] = src(*args[1], "SRC0")
            return
        if op in DIV_OPS:
            self._div_op(op, args, dr, src)
            return
        if op == "v_bitop3_b32":
            # bit i of the table is the result for sources (s0, s1, s2) = bits of i, s0 the highest
            A = src(*args[1], "SRC0").view(np.uint32)
            B = src(*args[2], "SRC1").view(np.uint32)
            Cc = src(*args[3], "SRC2").view(np.uint32)
            r = np.zeros(64, np.uint32)
            for i in range(8):
                if (args[4][1] >> i) & 1:
                    r |= (A if i & 4 else ~A) & (B if i & 2 else ~B) & (Cc if i & 1 else ~Cc)
            self.v[dr] = r.view(np.float32)
            return
        if op == "v_not_b32_e32":
            self.v[dr] = (~src(*args[1], "SRC0").view(np.uint32)).view(np.float32)
            return
        a = src(*args[1], "SRC0")
        b = src(*args[2], "SRC1")
        if op in ("v_and_b32_e32", "v_or_b32_e32"):
            ua, ub = a.view(np.uint32), b.view(np.uint32)
            self.v[dr] = ((ua & ub) if op == "v_and_b32_e32" else (ua | ub)).view(np.float32)
            return
        with np.errstate(all="ignore"):
            if op == "v_add_f32_e32": r = a + b
            elif op == "v_sub_f32_e32": r = a - b
            elif op == "v_subrev_f32_e32": r = b - a
            elif op == "v_mul_f32_e32": r = a * b
            else: raise AssertionError(op)
        self.v[dr] = r.astype(np.float32)

    def _div_op(self, op, args, dr, src):
        """The instructions of the division and classification handlers
        (compares into vcc or s[80:81], selects).  The scaling that
        v_div_scale / v_div_fmas apply near the ends of the exponent range is
        not modelled: the scale flag stays clear, and v_div_fixup gives the
        IEEE quotient wherever an operand or the result is zero, infinite,
        NaN or beyond 2^+-60 (where the hardware scales).  Elsewhere the
        quotient comes out of the reciprocal and its fused refinements, so
        operand offsets, the protection select and the destination are what
        is checked."""
        f64 = np.float64
        with np.errstate(all="ignore"):
            if op == "v_div_scale_f32":
                self.v[dr] = src(*args[2], "SRC0")
                self.vcc = np.zeros(64, bool)
            elif op == "v_rcp_f32_e32":
                self.v[dr] = (f64(1.0) / src(*args[1], "SRC0").astype(f64)).astype(np.float32)
            elif op in ("v_fma_f32", "v_div_fmas_f32"):
                a, b, c = src(*args[1], "SRC0"), src(*args[2], "SRC1"), src(*args[3], "SRC2")
                if op == "v_div_fmas_f32":
                    assert not self.vcc.any()
                self.v[dr] = (a.astype(f64) * b.astype(f64) + c.astype(f64)).astype(np.float32)
            elif op == "v_fmac_f32_e32":
                a, b = src(*args[1], "SRC0"), src(*args[2], "SRC1")
                self.v[dr] = (a.astype(f64) * b.astype(f64) + self.v[dr].astype(f64)).astype(np.float32)
            elif op == "v_div_fixup_f32":
                q, den, num = src(*args[1], "SRC0"), src(*args[2], "SRC1"), src(*args[3], "SRC2")
                ieee = (num.astype(f64) / den.astype(f64)).astype(np.float32)
                big = lambda x: ~np.isfinite(x) | (x == 0) | (np.abs(x) > 2.0 ** 60) | (np.abs(x) < 2.0 ** -60)
                self.v[dr] = np.where(big(num) | big(den) | big(q), ieee, q)
            elif op.startswith("v_cmp_"):
                a, b = src(*args[1], "SRC0"), src(*args[2], "SRC1")
                rel = op.split("_")[2]
                m = {"nlt": ~(a < b), "gt": a > b, "lt": a < b, "eq": a == b, "neq": ~(a == b)}[rel]
                if dr == "sp":
                    assert args[0][1] == 80
                    self.smask = m
                else:
                    self.vcc = m
            elif op in ("v_cndmask_b32_e32", "v_cndmask_b32_e64"):
                assert args[-1][0] == "vcc"
                a, b = src(*args[1], "SRC0"), src(*args[2], "SRC1")
                self.v[dr] = np.where(self.vcc, b, a)
            else:
                raise AssertionError(op)

    # ------------------------------------------------------------------ kernel side
    def gather(self, off):
        return self.v[self.V0 + off: self.V0 + off + self.T].copy()

    def scatter(self, off, vals):
        self.v[self.V0 + off: self.V0 + off + self.T] = vals

    def do_exit(self, pay, cst):
        """sin, cos, exp or log of the operand (or the constant), as the kernel's exit computes it."""
        oa, od = pay & 255, (pay >> 16) & 255
        op, fl = (pay >> 24) & 15, pay >> 28
        assert op in (synth.SIN, synth.COS, synth.EXPC, synth.PLOG), op
        c = np.frombuffer(np.uint32(cst).tobytes(), np.float32)[0]
        A = np.full((self.T, 64), c, np.float32) if fl & 1 else self.gather(oa)
        R = np.vectorize(lambda x: oracle.apply(op, x), otypes=[np.float32])(A)
        self.scatter(od, R.astype(np.float32))

    def evaluate(self, words, prog_off, X, n_load):
        T = self.T
        F, N = X.shape
        P = len(prog_off) - 1
        out = np.zeros((P, N), np.float32)
        lane = np.arange(64)
        for tile in range((N + 64 * T - 1) // (64 * T)):
            t0 = tile * 64 * T
            for f in range(n_load):
                vals = np.zeros((T, 64), np.float32)
                for j in range(T):
                    c = t0 + 64 * j + lane
                    ok = c < N
                    vals[j, ok] = X[f, c[ok]]
                self.scatter(self.FO + f * T, vals)
            for p in range(P):
                off = int(prog_off[p]) * 4
                while True:
                    off, pay, cst = self.run(words, off)
                    if (pay >> 24) & 15 == 15:
                        break
                    self.do_exit(pay, cst)
                    off += 16
                o = self.gather(0)
                for j in range(T):
                    c = t0 + 64 * j + lane
                    ok = c < N
                    out[p, c[ok]] = o[j, ok]
        return out


DIV_OPS = ("v_div_scale_f32", "v_rcp_f32_e32", "v_fma_f32", "v_div_fmas_f32", "v_fmac_f32_e32", "v_div_fixup_f32",
           "v_cmp_nlt_f32_e64", "v_cndmask_b32_e32", "v_cndmask_b32_e64") + tuple(
    "v_cmp_%s_f32_%s" % (r, e) for r in ("gt", "lt", "eq", "neq") for e in ("e32", "e64"))


def _same(a, b):
    return (a.view(np.int32) == b.view(np.int32)) | (np.isnan(a) & np.isnan(b))


REAL = [i for i, v in enumerate(gen_core.VARIANTS) if v[4] != 2]
LINEAR = [i for i, v in enumerate(gen_core.VARIANTS) if v[4] in (0, 1)]   # kernels with linear handlers
BOOL = [i for i, v in enumerate(gen_core.VARIANTS) if v[4] == 2]


@pytest.mark.parametrize("vi", REAL)
def test_core_trees_match_oracle(vi):
    T, D, NF, NCV = gen_core.VARIANTS[vi][:4]
    F = min(NF, 9)
    rng = synth.rng_for(300 + vi)
    pop = synth.ptc2_population(rng, 30, synth.FULL, F, 1, 90, 0.25)
    pop2 = synth.ramped_half_and_half(rng, 20, synth.ARITH3, F, 2, 5, 64, 0.2)
    pop3 = synth.trees_from_lists([
        (np.array([synth.var_tok(F - 1)], np.int32), np.zeros(1, np.float32)),      # lone variable
        (np.array([synth.CONST], np.int32), np.array([1.25], np.float32)),          # lone constant
        (np.array([synth.SUB, synth.CONST, synth.CONST], np.int32), np.array([0, 2, 0.5], np.float32)),
    ])
    pops = [pop, pop2, pop3]
    X = synth.uniform_cases(rng, F, 64 * T + 37, -3, 3)
    emu = CoreEmu(vi)
    for pp in pops:
        words, prog_off = gp.core_lower(pp, F, vi, BASE)
        n_load = F
        got = emu.evaluate(words, prog_off, X, n_load)
        ref = oracle.tree_outputs(pp.tok, pp.cst, pp.off, X)
        assert _same(got, ref).all()


@pytest.mark.parametrize("vi", [i for i in REAL if gen_core.VARIANTS[i][2] >= 9][:1] +
                         [i for i, v in enumerate(gen_core.VARIANTS) if v[4] in (3, 4) and v[2] >= 9])
def test_core_classification_match_oracle(vi):
    """Trees over the classification functions (comparisons, logical AND and
    OR, the three-operand IF; their terminal operands pushed at any level)
    run through the generated handlers and the kernel's exits to the
    oracle's bits."""
    T, D, NF, NCV = gen_core.VARIANTS[vi][:4]
    F = 9
    rng = synth.rng_for(500 + vi)
    pop = synth.ptc2_population(rng, 40, synth.SHUTTLE_SET, F, 1, 80, 0.2, crange=(-3.0, 3.0))
    X = np.round(synth.uniform_cases(rng, F, 64 * T + 11, -3, 3))
    emu = CoreEmu(vi)
    words, prog_off = gp.core_lower(pop, F, vi, BASE)
    got = emu.evaluate(words, prog_off, X, F)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert _same(got, ref).all()


@pytest.mark.parametrize("vi", [0] + [i for i, v in enumerate(gen_core.VARIANTS) if v[4] in (1, 3, 4)][:3])
def test_core_division_forms(vi):
    """Protected division runs in the core in every operand form: stack and
    stack in both orders, stack and variable, variable and stack, constants
    on either side, two variables, a variable and a constant, and the
    register forms; divisors below 1e-6 in magnitude (and zeros of both
    signs) give 1.  Every division handler is run, and the results are the
    oracle's bits."""
    T, D, NF, NCV, mode = gen_core.VARIANTS[vi]
    F = 3
    exprs = ["(/ x0 x1)", "(/ x1 x0)", "(/ (+ x0 x2) (* x1 x2))", "(/ (* x1 x2) (+ x0 x2))",
             "(/ (+ x0 x1) x2)", "(/ x2 (+ x0 x1))", "(/ (+ x0 x1) 0.37)", "(/ -2.5 (+ x0 x1))",
             "(/ x0 1e-7)", "(/ 3 x1)", "(/ x1 -0.0)", "(/ (/ x0 x1) (/ x2 (/ x1 x0)))",
             "(+ x0 (/ (- x1 x2) (* (+ x0 x0) (/ 1.5 x2))))"]
    from tests import progs
    pop = progs.pop(*exprs)
    rng = synth.rng_for(77)
    X = synth.uniform_cases(rng, F, 64 * T + 29, -3, 3)
    X[:, ::5] = 0.0
    X[1, 1::7] = -0.0
    X[1, 2::7] = 5e-7
    X[2, 3::11] = -9.9e-7
    X[0, 4::13] = 3.0e38
    emu = CoreEmu(vi)

    def handler_kinds(words):
        rec = words.reshape(-1, 4)
        out = []
        for r in rec:
            a = int(r[0]) | (int(r[1]) << 32)
            slot = (a - BASE) // gen_core.SLOT
            if a >= BASE and slot in emu.by_slot:
                out.append((emu.by_slot[slot].kind & 0x7F, int(r[2])))
        return out

    words, prog_off = gp.core_lower(pop, F, vi, BASE)
    got = emu.evaluate(words, prog_off, X, F)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert _same(got, ref).all(), np.argwhere(~_same(got, ref))[:4]
    hk = handler_kinds(words)
    for k in ("DVV", "DVC", "DCV"):
        assert any(kind == gen_core.K[k] for kind, _ in hk), k
    # no division leaves the core
    assert not any(kind == gen_core.K["EXIT"] and (pay >> 24) & 15 == synth.PDIV for kind, pay in hk)
    if mode in (0, 1):
        lp = synth.linear_population(rng, 12, 4, 40, (synth.PDIV, synth.ADD, synth.PDIV), 8, F, n_const=3,
                                     crange=(-2.0, 2.0))
        words, prog_off = gp.core_lower(lp, F, vi, BASE)
        got = emu.evaluate(words, prog_off, X, F)
        ref = oracle.linear_outputs(lp.code, lp.off, lp.cst, lp.cst_off, lp.n_reg, X)
        assert _same(got, ref).all()
        hk = handler_kinds(words)
        assert not any(kind == gen_core.K["EXIT"] and (pay >> 24) & 15 == synth.PDIV for kind, pay in hk)


@pytest.mark.parametrize("vi", [0] + [i for i, v in enumerate(gen_core.VARIANTS) if v[4] in (1, 3, 4)][:3])
def test_core_classification_forms(vi):
    """>, <, ==, AND, OR and IF run in the core in every operand form (two
    stack or feature operands, a constant on either side), with signed
    zeros, NaN and equal operands among the cases; only a function of two
    constants leaves the core.  Results are the oracle's bits."""
    T, D, NF, NCV, mode = gen_core.VARIANTS[vi]
    F = 3
    exprs = []
    for f in (">", "<", "==", "and", "or"):
        exprs += ["(%s x0 x1)" % f, "(%s x1 x0)" % f, "(%s (+ x0 x2) (* x1 x2))" % f, "(%s x2 0.5)" % f,
                  "(%s -0.0 x1)" % f, "(%s (- x0 x1) 0)" % f, "(%s 2 (* x0 x2))" % f, "(%s x0 x0)" % f]
    exprs += ["(if x0 x1 x2)", "(if (> x0 x1) (* x2 3) -1.5)", "(if 0 x0 x1)", "(if (and x0 x1) (or x1 x2) (== x0 x2))",
              "(if (if x0 x1 x2) (if x2 x1 x0) (+ x0 (if x1 1 2)))", "(> 1 2)"]
    from tests import progs
    pop = progs.pop(*exprs)
    rng = synth.rng_for(78)
    X = np.round(synth.uniform_cases(rng, F, 64 * T + 19, -2, 2))
    X[0, ::7] = -0.0
    X[1, 1::9] = np.nan
    X[2, 2::11] = np.inf
    X[1, 3::5] = X[0, 3::5]
    emu = CoreEmu(vi)
    words, prog_off = gp.core_lower(pop, F, vi, BASE)
    got = emu.evaluate(words, prog_off, X, F)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert _same(got, ref).all(), np.argwhere(~_same(got, ref))[:4]
    kinds = []
    for r in words.reshape(-1, 4):
        a = int(r[0]) | (int(r[1]) << 32)
        slot = (a - BASE) // gen_core.SLOT
        if a >= BASE and slot in emu.by_slot:
            kinds.append((emu.by_slot[slot].kind & 0x7F, int(r[2])))
    for k in ("CVV", "CVC", "CCV", "IF3"):
        assert any(kind == gen_core.K[k] for kind, _ in kinds), k
    leaving = [(pay >> 24) & 15 for kind, pay in kinds if kind == gen_core.K["EXIT"] and (pay >> 24) & 15 != 15]
    assert leaving == [], leaving


@pytest.mark.parametrize("vi", LINEAR)
def test_core_linear_match_oracle(vi):
    T, D, NF, NCV = gen_core.VARIANTS[vi][:4]
    F = min(NF, 12)
    rng = synth.rng_for(400 + vi)
    pop = synth.linear_population(rng, 25, 1, 60, synth.FULL, 8, F, n_const=3)
    pop_b = synth.linear_population(rng, 10, 1, 40, synth.BASIC, 5, F, n_const=2)
    X = synth.uniform_cases(rng, F, 64 * T + 5, -3, 3)
    emu = CoreEmu(vi)
    for pp in (pop, pop_b):
        words, prog_off = gp.core_lower(pp, F, vi, BASE)
        got = emu.evaluate(words, prog_off, X, F)
        ref = oracle.linear_outputs(pp.code, pp.off, pp.cst, pp.cst_off, pp.n_reg, X)
        assert _same(got, ref).all()


@pytest.mark.parametrize("vi", BOOL)
def test_core_bool_match_oracle(vi):
    # Boolean kernels: slots are 32-bit words of bit-packed cases; the core's
    # output words must equal the oracle's bit for bit
    from tests import boolprogs as bp
    T, D, NF, NCV, _ = gen_core.VARIANTS[vi]
    F = min(NF, 20)
    rng = synth.rng_for(500 + vi)
    pop = synth.ptc2_population(rng, 30, synth.BOOL_SET, F, 1, 120, 0.0)
    sol = bp.mux_solution(2)
    x = bp.var(F - 1)
    pop2 = bp.pop_of(sol, x, bp.NOT(x), bp.fn(synth.NOR, x, bp.var(0)), bp.fn(synth.NAND, bp.var(1), bp.var(0)))
    W = 64 * T + 37
    Xw = rng.integers(0, 2**32, size=(F, W), dtype=np.uint64).astype(np.uint32)
    emu = CoreEmu(vi)
    for pp in (pop, pop2):
        words, prog_off = gp.core_lower(pp, F, vi, BASE)
        got = emu.evaluate(words, prog_off, Xw.view(np.float32), F).view(np.uint32)
        ref = oracle.bool_outputs(pp.tok, pp.off, Xw)
        assert (got == ref).all()


def test_every_handler_is_reachable_and_in_its_slot():
    for vi, (T, D, NF, NCV, mode) in enumerate(gen_core.VARIANTS):
        tag, V0, FO, hs, nslots = gen_core.gen_variant(T, D, NF, NCV, mode)
        slots = [h.slot for h in hs]
        assert slots == sorted(slots) and len(set(slots)) == len(slots)
        for h in hs:
            assert h.size <= gen_core.SLOT * ((h.size + gen_core.SLOT - 1) // gen_core.SLOT)
            if h.kind & 0x7F == gen_core.K["EXIT"]:
                continue
            if h.kind & gen_core.PHASE_B:
                # loads the next two records, waits, jumps to the first of them
                assert h.lines[-1] == "s_setpc_b64 s[64:65]" and h.lines[-2] == "s_waitcnt lgkmcnt(0)"
                loads = [i for i, x in enumerate(h.lines) if x.startswith("s_load_dwordx8")]
                assert len(loads) == 1
                # everything read from its own record (s[68:71]) is read before the load
                assert not any(re.search(r"\bs(68|69|70|71)\b", x) for x in h.lines[loads[0] + 1:])
            else:
                # works from s[64:67] and jumps to the record already in s[68:69]
                assert h.lines[-1] == "s_setpc_b64 s[68:69]"
                assert not any(x.startswith(("s_load", "s_waitcnt")) for x in h.lines)
        assert V0 + FO + NF * T <= 256
