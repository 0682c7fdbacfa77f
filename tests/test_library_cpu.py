"""Host-side checks of libgp.so that need no GPU: the library loads, exports
every entry point include/gp.h declares, validates programs, and its tree
lowering preserves each program's value and bounds the stack depth."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests import progs

HERE = os.path.dirname(os.path.abspath(__file__))


def declared_functions():
    src = open(gp.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*\b(gp_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "gp_eval_tree" in names and "gp_eval_linear" in names
    L = ctypes.CDLL(gp.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert gp.version().startswith("gp2d")


def test_worked_example_lowering_counts():
    g = json.load(open(os.path.join(HERE, "golden", "sextic_worked_example.json")))
    tok, cst = progs.parse(g["prefix"])
    words, st = gp.gp_lower_tree(tok, cst, 1)
    assert st["n_nodes"] == g["rpn"]["tokens"]
    assert st["n_instr"] == g["lgp"]["instructions"]
    assert st["n_values"] == g["lgp"]["values"]
    assert st["stack_fetches"] == g["lgp"]["stack_fetches"]
    assert st["max_depth"] == g["lgp"]["max_depth"]


# --- a test-side reader of the lowered words, to check the lowering on the CPU
MODES = dict(SS=0, SSR=1, SX=2, XS=3, SC=4, CS=5, XX=6, XC=7, CX=8, S=9, X=10, C=11, S3=12)
OP_IF = 10     # the three-operand IF in a lowered word


def run_lowered(words, X):
    """Evaluate lowered words on every case with numpy float32 arithmetic
    (+ - * /p and the classification functions; transcendentals are not used
    with this reader)."""
    F, N = X.shape
    st = []
    w = words.reshape(-1, 2)
    t = lambda m: m.astype(np.float32)
    for w0, w1 in w:
        op, mode, fa, fb, hafter = w0 & 15, (w0 >> 4) & 15, (w0 >> 8) & 255, (w0 >> 16) & 255, w0 >> 24
        c = np.frombuffer(np.uint32(w1).tobytes(), np.float32)[0]
        cv = np.full(N, c, np.float32)
        if mode == 12:
            assert op == OP_IF
            three = st[-3:]
            del st[-3:]
            A, B, C = three[fa], three[fb], three[3 - fa - fb]
            st.append(np.where(A != 0, B, C).astype(np.float32))
            assert len(st) == hafter
            continue
        if mode in (0, 1):
            b2, b1 = st.pop(), st.pop()
            A, B = (b1, b2) if mode == 0 else (b2, b1)
        elif mode == 2: A, B = st.pop(), X[fb]
        elif mode == 3: A, B = X[fa], st.pop()
        elif mode == 4: A, B = st.pop(), cv
        elif mode == 5: A, B = cv, st.pop()
        elif mode == 6: A, B = X[fa], X[fb]
        elif mode == 7: A, B = X[fa], cv
        elif mode == 8: A, B = cv, X[fb]
        elif mode == 10: A, B = X[fa], None
        elif mode == 11: A, B = cv, None
        else: raise AssertionError("unexpected mode")
        with np.errstate(all="ignore"):
            if op == 0: R = A + B
            elif op == 1: R = A - B
            elif op == 2: R = A * B
            elif op == 3: R = np.where(np.abs(B) < np.float32(1e-6), np.float32(1), A / B)
            elif op == 8: R = t((A != 0) & (B != 0))
            elif op == 9: R = t((A != 0) | (B != 0))
            elif op == 12: R = t(A > B)
            elif op == 13: R = t(A < B)
            elif op == 14: R = t(A == B)
            elif op == 15: R = A          # push
            else: raise AssertionError("op")
        st.append(R.astype(np.float32))
        assert len(st) == hafter
    assert len(st) == 1
    return st[0]


def test_lowering_preserves_values_bit_exact():
    rng = synth.rng_for(5)
    pop = synth.ptc2_population(rng, 300, synth.BASIC, 4, 1, 120, 0.3)
    X = synth.uniform_cases(rng, 4, 37, -3, 3)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    nrev = 0
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        words, st = gp.gp_lower_tree(t, c, 4)
        nrev += st["n_reversed"]
        got = run_lowered(words, X)
        same = (got.view(np.int32) == ref[p].view(np.int32)) | (np.isnan(got) & np.isnan(ref[p]))
        assert same.all(), p
    assert nrev > 0   # the reversed (right-first) operand order was exercised


def test_lowering_classification_trees_bit_exact():
    """Trees over the classification set (>, <, ==, AND, OR, IF and + - * /)
    lower to words that the test-side reader evaluates to the oracle's bits:
    IF's operands run in order of decreasing need and are read from where
    they landed on the stack."""
    rng = synth.rng_for(15)
    pop = synth.ptc2_population(rng, 300, synth.SHUTTLE_SET, 5, 1, 150, 0.2, crange=(-3.0, 3.0))
    X = np.round(synth.uniform_cases(rng, 5, 41, -3, 3))      # small integers: comparisons often tie
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    n_if = 0
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        words, st = gp.gp_lower_tree(t, c, 5)
        n_if += int(np.sum((t & 0xFF) == synth.IF))
        got = run_lowered(words, X)
        same = (got.view(np.int32) == ref[p].view(np.int32)) | (np.isnan(got) & np.isnan(ref[p]))
        assert same.all(), p
        # every IF reads three stack values; its terminal operands are pushed
        assert st["n_values"] == sum(1 + synth.ARITY[int(o)] for o in (t & 0xFF) if int(o) < 64)
    assert n_if > 100


def test_lowering_depth_bound():
    rng = synth.rng_for(6)
    pop = synth.ptc2_population(rng, 400, synth.FULL, 8, 1, 256, 1 / 9)
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        _, st = gp.gp_lower_tree(t, c, 8)
        n_term = int(np.sum((t & 0xFF) >= 64))
        assert st["max_depth"] <= int(np.floor(np.log2(max(n_term, 1)))) + 1
        n_fun = st["n_nodes"] - n_term
        n_const = int(np.sum((t & 0xFF) == synth.CONST))
        # one instruction per function, plus one push per function whose two
        # operands are both constants (or for a lone terminal)
        assert n_fun <= st["n_instr"] <= max(n_fun + n_const // 2, 1)


def test_comb_lowers_to_depth_one():
    e = "x0"
    for _ in range(127):
        e = "(+ x0 %s)" % e
    tok, cst = progs.parse(e)
    _, st = gp.gp_lower_tree(tok, cst, 1)
    assert st["max_depth"] == 1 and st["n_instr"] == 127


def test_deepest_trees_lower():
    """The largest full binary tree within GP_MAX_LEN needs 15 levels; an
    IF-rich tree of 59,050 nodes needs 20, the limit, so every valid tree
    lowers (no depth rejection below GP_MAX_LEN nodes)."""
    from tests import deeptrees
    t = deeptrees.Tree(synth.rng_for(3), 1)
    t.full(15)
    tok, cst = t.lists()
    assert len(tok) == 65535
    _, st = gp.gp_lower_tree(tok, cst, 1)
    assert st["max_depth"] == 15
    tok, cst = deeptrees.need20(synth.rng_for(4), 3)
    assert len(tok) == 59050
    _, st = gp.gp_lower_tree(tok, cst, 3)
    assert st["max_depth"] == gp.GP_MAX_DEPTH == 20
    t = deeptrees.Tree(synth.rng_for(5), 2)
    t.full_if(6)                          # 1,093 nodes, 13 levels
    tok, cst = t.lists()
    _, st = gp.gp_lower_tree(tok, cst, 2)
    assert (len(tok), st["max_depth"]) == (1093, 13)


def test_smallest_tree_per_depth_brute_force():
    """The growth that bounds the depth at 20: the fewest nodes of a tree
    needing k levels, by exhaustive search over shapes up to 28 nodes (with
    unary, binary and IF functions), equals the recurrence
    m(k) = min(2 m(k-1) + 1, 3 m(k-2) + 1) that the deep trees follow."""
    from functools import lru_cache
    import itertools

    @lru_cache(None)
    def needs(n):
        """Set of (need, is_terminal) reachable by trees of exactly n nodes."""
        if n == 1:
            return frozenset({(1, True)})
        r = set()
        for a in needs(n - 1):                 # unary
            r.add((a[0], False))
        for k in range(1, n - 1):              # binary: k + (n-1-k) nodes
            for a in needs(k):
                for b in needs(n - 1 - k):
                    if a[1] and b[1]:
                        r.add((1, False))
                    elif b[1]:
                        r.add((a[0], False))
                    elif a[1]:
                        r.add((b[0], False))
                    else:
                        r.add((max(a[0], b[0]) if a[0] != b[0] else a[0] + 1, False))
        for i in range(1, n - 2):              # IF: three operands
            for j in range(1, n - 1 - i):
                k = n - 1 - i - j
                if k < 1:
                    continue
                for a, b, c in itertools.product(needs(i), needs(j), needs(k)):
                    nd = sorted([a[0], b[0], c[0]], reverse=True)
                    r.add((max(nd[0], nd[1] + 1, nd[2] + 2), False))
        return frozenset(r)

    exact = {}
    for n in range(1, 29):
        for d, term in needs(n):
            if not term:
                exact.setdefault(d, n)
    fewest = {k: min(n for d, n in exact.items() if d >= k) for k in exact}   # needing at least k
    m = {1: 2, 2: 4, 3: 4}
    for k in range(4, 22):
        m[k] = min(2 * m[k - 1] + 1, 3 * m[k - 2] + 1)
    assert len(fewest) == 6 and all(fewest[k] == m[k] for k in fewest), (fewest, m)
    assert m[20] <= 65536 < m[21]
    import re
    hdr = open(gp.HEADER).read()
    for name in ("GP_MAX_DEPTH", "GP_MAX_LEN", "GP_MAX_FEAT"):
        assert int(re.search(r"#define %s (\d+)" % name, hdr).group(1)) == getattr(gp, name)
    assert m[gp.GP_MAX_DEPTH] <= gp.GP_MAX_LEN < m[gp.GP_MAX_DEPTH + 1]


@pytest.mark.parametrize("tok", [
    [synth.ADD, synth.var_tok(0)],                 # missing operand
    [synth.var_tok(0), synth.var_tok(0)],          # trailing token
    [synth.var_tok(3)],                            # feature out of range
    [99],                                          # unknown opcode
    [synth.CONST | (1 << 8)],                      # stray argument bits
])
def test_lowering_rejects_malformed(tok):
    with pytest.raises(gp.GPError) as e:
        gp.gp_lower_tree(np.array(tok, np.int32), np.zeros(len(tok), np.float32), 2)
    assert e.value.status == gp.GP_E_INVAL


def test_eval_rejects_malformed_before_touching_the_device():
    L = gp.lib()
    tok = np.array([synth.ADD, synth.var_tok(0)], np.int32)
    cst = np.zeros(2, np.float32)
    off = np.array([0, 2], np.int64)
    rc = L.gp_eval_tree(tok.ctypes.data, cst.ctypes.data, off.ctypes.data, 1, None, 1, 10, None, 0, None, None)
    assert rc == gp.GP_E_INVAL and "unfilled" in gp.last_error()
    code = np.array([synth.lin_word(synth.ADD, 9, 0, 0)], np.uint32)
    rc = L.gp_eval_linear(code.ctypes.data, off[:2].ctypes.data, None, None, 1, 8, None, 1, 10, None, 2, None, None)
    assert rc == gp.GP_E_INVAL and "dst" in gp.last_error()
    code = np.array([synth.lin_word(synth.ADD, 0, 0, 200)], np.uint32)
    rc = L.gp_eval_linear(code.ctypes.data, off[:2].ctypes.data, None, None, 1, 8, None, 4, 10, None, 2, None, None)
    assert rc == gp.GP_E_INVAL and "source" in gp.last_error()
    rc = L.gp_eval_linear(code.ctypes.data, off[:2].ctypes.data, None, None, 1, 9, None, 4, 10, None, 2, None, None)
    assert rc == gp.GP_E_INVAL and "n_reg" in gp.last_error()


def test_zero_programs_is_a_no_op():
    L = gp.lib()
    off = np.zeros(1, np.int64)
    assert L.gp_eval_tree(None, None, off.ctypes.data, 0, None, 1, 10, None, 0, None, None) == 0
