"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints for its worked example, closed forms, algebraic identities, IEEE
binary32 arithmetic as numpy implements it, high-precision values from mpmath,
and brute-force agreement between structurally different interpreters.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
import synth
from tests import progs

HERE = os.path.dirname(os.path.abspath(__file__))
f32 = np.float32


def one(expr, X, kind="cases", y=None):
    p = progs.pop(expr)
    return oracle.eval_tree(p.tok, p.cst, p.off, X, y, kind)


def ulp_dist(a, b):
    """Distance in representable binary32 steps (NaN==NaN counts as 0)."""
    a = np.asarray(a, np.float32); b = np.asarray(b, np.float32)
    ia = a.view(np.int32).astype(np.int64); ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    d = np.abs(ia - ib)
    both_nan = np.isnan(a) & np.isnan(b)
    return np.where(both_nan, 0, d)


# --------------------------------------------------------------------------
# Hand-computed programs (exact binary32 results)
# --------------------------------------------------------------------------
def test_hand_computed_values():
    X = np.array([[0.25]], np.float32)
    assert one("(+ (* x0 x0) 0.5)", X)[0, 0] == f32(0.5625)
    assert one("(/ 3 2)", X)[0, 0] == f32(1.5)
    assert one("(/ x0 0)", X)[0, 0] == f32(1.0)            # protected: |b| < 1e-6
    assert one("(/ 1 5e-7)", X)[0, 0] == f32(1.0)          # protected
    # 1e-6f is not below itself: the division happens (threshold compared in binary32)
    assert one("(/ 1 1e-6)", X)[0, 0] == f32(1.0) / f32(1e-6)
    assert one("(/ 1 1e-6)", X)[0, 0] == f32(1e6)
    assert one("(- x0 (* x0 4))", X)[0, 0] == f32(-0.75)
    assert one("(log 5e-7)", X)[0, 0] == f32(0.0)           # protected log
    assert one("(exp 1000)", X)[0, 0] == one("(exp 88)", X)[0, 0]
    assert np.isfinite(one("(exp 1000)", X)[0, 0])


def test_protected_ops_special_values():
    nan, inf = np.float32(np.nan), np.float32(np.inf)
    assert np.isnan(oracle.apply(synth.PDIV, 1.0, nan))
    assert oracle.apply(synth.PDIV, nan, 0.0) == f32(1.0)
    assert oracle.apply(synth.PDIV, 1.0, -1e-7) == f32(1.0)
    assert oracle.apply(synth.PDIV, 0.0, inf) == f32(0.0)
    assert np.isnan(oracle.apply(synth.PLOG, nan))
    assert oracle.apply(synth.PLOG, inf) == inf
    assert oracle.apply(synth.PLOG, -1.0) == f32(0.0)
    assert np.isnan(oracle.apply(synth.EXPC, nan))       # NaN passes the clamp
    assert oracle.apply(synth.EXPC, -inf) == f32(0.0)
    assert oracle.apply(synth.EXPC, inf) == oracle.apply(synth.EXPC, 88.0)
    assert np.isnan(oracle.apply(synth.SIN, inf))
    assert np.isnan(oracle.apply(synth.COS, -inf))


# --------------------------------------------------------------------------
# Identities (hold for every finite input)
# --------------------------------------------------------------------------
def test_identities():
    rng = synth.rng_for(101)
    x = rng.uniform(-1e4, 1e4, size=(1, 4096)).astype(np.float32)
    x[0, :8] = [0.0, -0.0, 1e-30, -1e-30, 3e-39, 1.0, -1.0, 2.5]
    assert np.all(one("(- (* x0 x0) (* x0 x0))", x) == 0.0)
    assert not np.any(np.signbit(one("(- (* x0 x0) (* x0 x0))", x)))
    r = one("(/ x0 x0)", x)
    assert np.all(r == 1.0)                         # both branches give 1
    assert np.all(one("(- x0 x0)", x) == 0.0)
    assert np.array_equal(one("(* x0 1)", x)[0].view(np.int32), x[0].view(np.int32))
    assert one("(log 1)", x)[0, 0] == 0.0
    assert one("(sin 0)", x)[0, 0] == 0.0
    assert one("(cos 0)", x)[0, 0] == 1.0
    assert one("(exp 0)", x)[0, 0] == 1.0
    # odd / even symmetry of the binary64-rounded functions
    xs = x[0]
    s1 = oracle.tree_outputs(*_arrs("(sin x0)"), x)[0]
    s2 = oracle.tree_outputs(*_arrs("(sin (- 0 x0))"), x)[0]
    assert np.array_equal(s1[xs != 0], -s2[xs != 0])
    c1 = oracle.tree_outputs(*_arrs("(cos x0)"), x)[0]
    c2 = oracle.tree_outputs(*_arrs("(cos (- 0 x0))"), x)[0]
    assert np.array_equal(c1, c2)
    # log|a| is even in a
    l1 = oracle.tree_outputs(*_arrs("(log x0)"), x)[0]
    l2 = oracle.tree_outputs(*_arrs("(log (- 0 x0))"), x)[0]
    assert np.array_equal(l1, l2)


def _arrs(e):
    p = progs.pop(e)
    return p.tok, p.cst, p.off


# --------------------------------------------------------------------------
# IEEE binary32 arithmetic: + - * / are correctly rounded, so numpy's
# float32 operators define the unique right answer.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("op,npop", [(synth.ADD, np.add), (synth.SUB, np.subtract),
                                      (synth.MUL, np.multiply)])
def test_basic_ops_match_ieee(op, npop):
    rng = synth.rng_for(7)
    a = (rng.standard_normal(3000) * 10.0 ** rng.integers(-40, 38, 3000)).astype(np.float32)
    b = (rng.standard_normal(3000) * 10.0 ** rng.integers(-40, 38, 3000)).astype(np.float32)
    with np.errstate(all="ignore"):
        ref = npop(a, b).astype(np.float32)
    got = oracle.apply_vec(op, a, b)
    assert np.array_equal(got.view(np.int32), ref.view(np.int32))


def test_pdiv_matches_ieee_and_threshold():
    rng = synth.rng_for(8)
    a = (rng.standard_normal(3000) * 10.0 ** rng.integers(-20, 20, 3000)).astype(np.float32)
    b = (rng.standard_normal(3000) * 10.0 ** rng.integers(-9, 9, 3000)).astype(np.float32)
    with np.errstate(all="ignore"):
        ref = np.where(np.abs(b) < np.float32(1e-6), np.float32(1.0), (a / b).astype(np.float32))
    got = oracle.apply_vec(synth.PDIV, a, b)
    assert np.array_equal(got.view(np.int32), ref.astype(np.float32).view(np.int32))
    t = np.float32(1e-6)
    below = np.nextafter(t, np.float32(0))
    assert oracle.apply(synth.PDIV, 2.0, below) == 1.0
    assert oracle.apply(synth.PDIV, 2.0, -below) == 1.0
    assert oracle.apply(synth.PDIV, 2.0, t) == np.float32(2.0) / t


# --------------------------------------------------------------------------
# Transcendentals against mpmath at 60 digits, rounded to binary32.
# The oracle rounds a binary64 result once, so it is within one step of the
# correctly rounded value.
# --------------------------------------------------------------------------
def _mp_ref(op, x):
    mpmath.mp.dps = 60
    v = mpmath.mpf(float(x))
    if op == synth.SIN:
        r = mpmath.sin(v)
    elif op == synth.COS:
        r = mpmath.cos(v)
    elif op == synth.EXPC:
        r = mpmath.exp(min(v, mpmath.mpf(88)))
    else:
        if abs(v) < mpmath.mpf(float(np.float32(1e-6))):
            return np.float32(0.0)
        r = mpmath.log(abs(v))
    return np.float32(float(r))


@pytest.mark.parametrize("op", [synth.SIN, synth.COS, synth.EXPC, synth.PLOG])
def test_transcendentals_against_mpmath(op):
    rng = synth.rng_for(11 + op)
    xs = np.concatenate([
        rng.uniform(-10, 10, 300),
        rng.standard_normal(100) * 1e3,
        10.0 ** rng.uniform(-30, 30, 100) * rng.choice([-1, 1], 100),
        np.array([0.0, 1e-7, 1.0, -1.0, 88.0, 87.9, 100.0, 1e4, 3e38, math.pi]),
    ]).astype(np.float32)
    if op == synth.EXPC:
        xs = xs[xs < 1e30]
    got = oracle.apply_vec(op, xs)
    ref = np.array([_mp_ref(op, x) for x in xs], np.float32)
    d = ulp_dist(got, ref)
    assert d.max() <= 1, (xs[d.argmax()], got[d.argmax()], ref[d.argmax()])


# --------------------------------------------------------------------------
# The paper's worked example (section 5, Figure 2): counts of the postfix
# and linear forms, and the value of the tree against its closed form.
# --------------------------------------------------------------------------
def test_worked_example_counts():
    g = json.load(open(os.path.join(HERE, "golden", "sextic_worked_example.json")))
    tok, cst = progs.parse(g["prefix"])
    rt, rc = oracle.prefix_to_rpn(tok, cst)
    assert len(rt) == g["rpn"]["tokens"]
    assert sum(1 for t in rt if (t & 0xFF) < 64) == g["rpn"]["functions"]
    X = np.array([[0.7]], np.float32)
    v, depth, fetch = oracle.rpn_eval(rt, rc, X, 0)
    assert depth == g["rpn"]["max_depth"]
    assert fetch == g["rpn"]["stack_fetches"]
    ins, m = oracle.rpn_to_lgp(rt, rc)
    assert m == g["lgp"]["instructions"]
    values = sum(1 + ins[i].n_args for i in range(m))
    assert values == g["lgp"]["values"]
    kinds = ["".join("SXC"[ins[i].kind[k]] for k in range(ins[i].n_args)) for i in range(m)]
    assert kinds == g["lgp"]["operand_kinds"]
    v2, d2, f2 = oracle.lgp_eval(ins, m, X, 0)
    assert d2 == g["lgp"]["max_depth"]
    assert f2 == g["lgp"]["stack_fetches"]
    assert v2 == v


def test_worked_example_closed_form():
    g = json.load(open(os.path.join(HERE, "golden", "sextic_worked_example.json")))
    xs = np.linspace(-1, 1, 2001).astype(np.float32)[None, :]
    got = one(g["prefix"], xs)[0].astype(np.float64)
    x = xs[0].astype(np.float64)
    exact = x ** 6 - 2 * x ** 4 + x ** 2
    # forward error of (x*(x*x) - x)^2 in binary32 for |x| <= 1 is below 7 units of 2^-24
    assert np.max(np.abs(got - exact)) <= 7 * 2.0 ** -24
    # a program evaluated against targets it generated has zero error
    y = one(g["prefix"], xs)[0]
    assert one(g["prefix"], xs, "mse", y)[0] == 0.0
    assert one(g["prefix"], xs, "sum_abs", y)[0] == 0.0


def test_wrong_inner_operator_is_not_the_sextic():
    # the printed postfix string, read literally, is (2x^2 - x)^2
    xs = np.array([[0.5]], np.float32)
    lit = one("(* (- (* x0 (+ x0 x0)) x0) (- (* x0 (+ x0 x0)) x0))", xs)[0, 0]
    assert lit == f32((2 * 0.25 - 0.5) ** 2)
    assert lit != one("(* (- (* x0 (* x0 x0)) x0) (- (* x0 (* x0 x0)) x0))", xs)[0, 0]


# --------------------------------------------------------------------------
# Structurally different interpreters agree bit for bit: recursive prefix,
# postfix one-dimensional stack, and the paper's stack-operand linear form.
# --------------------------------------------------------------------------
def test_recursive_rpn_lgp_agree():
    rng = synth.rng_for(21)
    pop = synth.ptc2_population(rng, 120, synth.FULL, 3, 1, 60, 0.25)
    X = synth.uniform_cases(rng, 3, 16, -3, 3)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        rt, rc = oracle.prefix_to_rpn(t, c)
        ins, m = oracle.rpn_to_lgp(rt, rc)
        for cc in range(X.shape[1]):
            v1, d1, _ = oracle.rpn_eval(rt, rc, X, cc)
            assert v1.view(np.int32) == ref[p, cc].view(np.int32) or (np.isnan(v1) and np.isnan(ref[p, cc]))
            if m:
                v2, d2, _ = oracle.lgp_eval(ins, m, X, cc)
                assert v2.view(np.int32) == v1.view(np.int32) or (np.isnan(v1) and np.isnan(v2))
                assert d2 <= d1


def test_right_comb_depth():
    # (+ x0 (+ x0 (+ x0 ... x0))) with 255 nodes needs a postfix stack of 128
    e = "x0"
    for _ in range(127):
        e = "(+ x0 %s)" % e
    tok, cst = progs.parse(e)
    assert len(tok) == 255
    rt, rc = oracle.prefix_to_rpn(tok, cst)
    v, depth, fetch = oracle.rpn_eval(rt, rc, np.array([[1.0]], np.float32), 0)
    assert depth == 128 and v == 128.0 and fetch == 254


# --------------------------------------------------------------------------
# Fitness closed forms
# --------------------------------------------------------------------------
def test_fitness_closed_forms():
    X = np.linspace(-1, 1, 1024).astype(np.float32)[None, :]
    y0 = np.zeros(1024, np.float32)
    assert one("0.5", X, "sum_abs", y0)[0] == 512.0
    assert one("0.5", X, "mse", y0)[0] == 0.25
    assert one("x0", X, "mse", X[0])[0] == 0.0
    assert one("x0", X, "sum_abs", X[0])[0] == 0.0
    ypos = np.where(np.arange(1024) % 3 == 0, 1.0, -1.0).astype(np.float32)
    assert one("1", X, "hits", ypos)[0] == int((ypos > 0).sum())
    assert one("-1", X, "hits", ypos)[0] == int((ypos <= 0).sum())
    # NaN output is never a hit and makes the error sums NaN
    assert one("(log (- x0 x0))", X, "hits", ypos)[0] == int((ypos <= 0).sum())  # log 0 -> 0
    assert np.isnan(one("(* (exp 88) (exp 88))", X, "mse", y0)[0]) is np.False_
    assert np.isinf(one("(* (exp 88) (exp 88))", X, "mse", y0)[0])
    assert np.isnan(one("(sin (* (exp 88) (exp 88)))", X, "mse", y0)[0])


# --------------------------------------------------------------------------
# Register linear GP
# --------------------------------------------------------------------------
def _lin(codes, consts=None, R=8):
    consts = consts or [np.zeros(0, np.float32)] * len(codes)
    return synth.linear_from_lists(codes, consts, R)


def test_linear_hit_pin_replays_label_model():
    rng = synth.rng_for(31)
    F, N, R = 16, 4096, 8
    X = synth.normal_cases(rng, F, N)
    w, y = synth.sign_labels(rng, X)
    # r0 = w0*x0; then r1 = wf*xf; r0 = r0 + r1  (the same binary32 sequence)
    code = [synth.lin_word(synth.MUL, 0, 128, R + 0, )]
    for f in range(1, F):
        code.append(synth.lin_word(synth.MUL, 1, 128 + f, R + f))
        code.append(synth.lin_word(synth.ADD, 0, 0, 1))
    neg = code + [synth.lin_word(synth.SUB, 0, 2, 0)]     # r2 is rewritten below
    neg = code + [synth.lin_word(synth.MUL, 2, 0, 0), synth.lin_word(synth.SUB, 2, 2, 2),
                  synth.lin_word(synth.SUB, 0, 2, 0)]     # r0 = 0 - r0 (r2 = r0*r0 - r0*r0 = 0)
    pop = _lin([np.array(code, np.uint32), np.array(neg, np.uint32)], [w, w], R)
    hits = oracle.eval_linear(pop.code, pop.off, pop.cst, pop.cst_off, R, X, y, "hits")
    assert hits[0] == N
    assert hits[1] == 0


def test_linear_register_init_and_unary():
    F, R = 3, 8
    X = np.array([[1.0, 2.0], [10.0, 20.0], [100.0, 200.0]], np.float32)
    # r0 starts as x0; r5 starts as x(5 mod 3) = x2
    code = [synth.lin_word(synth.ADD, 0, 0, 5)]
    # unary reads src1 only: src2 holds an out-of-range id that must be ignored
    code2 = [synth.lin_word(synth.SIN, 0, 3, 250)]
    pop = _lin([np.array(code, np.uint32), np.array(code2, np.uint32)], None, R)
    out = oracle.linear_outputs(pop.code, pop.off, pop.cst, pop.cst_off, R, X)
    assert np.array_equal(out[0], np.array([101.0, 202.0], np.float32))
    assert out[1, 0] == oracle.apply(synth.SIN, 1.0)      # id 3 = register r3 = x0


def test_tree_and_linear_agree():
    rng = synth.rng_for(41)
    F, R = 4, 8
    pop = synth.ptc2_population(rng, 150, synth.FULL, F, 2, 80, 0.2)
    X = synth.uniform_cases(rng, F, 64, -4, 4)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    codes, consts, keep = [], [], []
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        r = progs.tree_to_register_lgp(t, c, R)
        if r is None:
            continue
        codes.append(r[0]); consts.append(r[1]); keep.append(p)
    assert len(keep) > 100
    lp = _lin(codes, consts, R)
    out = oracle.linear_outputs(lp.code, lp.off, lp.cst, lp.cst_off, R, X)
    a = out.view(np.int32); b = ref[keep].view(np.int32)
    same = (a == b) | (np.isnan(out) & np.isnan(ref[keep]))
    assert same.all()


def test_multithreaded_equals_single():
    w = synth.tiny_tree_workload(1, 40, 300)
    y = w.X[0] * 0.5
    a = oracle.eval_tree(w.pop.tok, w.pop.cst, w.pop.off, w.X, y, "sum_abs", threads=1)
    b = oracle.eval_tree(w.pop.tok, w.pop.cst, w.pop.off, w.X, y, "sum_abs", threads=4)
    assert np.array_equal(a, b)


def test_nudge_moves_only_transcendentals():
    X = np.array([[0.3, 2.0]], np.float32)
    p = progs.pop("(+ x0 x0)", "(sin x0)")
    a = oracle.tree_outputs(p.tok, p.cst, p.off, X, nudge=0)
    b = oracle.tree_outputs(p.tok, p.cst, p.off, X, nudge=2)
    assert np.array_equal(a[0], b[0])
    assert np.all(ulp_dist(a[1], b[1]) == 2)


def test_malformed_rejected():
    with pytest.raises(ValueError):
        oracle.tree_outputs(np.array([synth.ADD, synth.var_tok(0)], np.int32),
                            np.zeros(2, np.float32), np.array([0, 2]), np.zeros((1, 4), np.float32))
    with pytest.raises(ValueError):
        oracle.tree_outputs(np.array([synth.var_tok(5)], np.int32), np.zeros(1, np.float32),
                            np.array([0, 1]), np.zeros((1, 4), np.float32))


# --------------------------------------------------------------------------
# Classification functions (section 4.2: >, <, ==, AND, OR, IF) and the
# classification fitness (Table 2: the sum of incorrect classifications)
# --------------------------------------------------------------------------
NAN = float("nan")


@pytest.mark.parametrize("op,cases", [
    (synth.GT, [(2, 1, 1), (1, 2, 0), (1, 1, 0), (-0.0, 0.0, 0), (NAN, 0, 0), (0, NAN, 0), (math.inf, 1e38, 1)]),
    (synth.LT, [(2, 1, 0), (1, 2, 1), (1, 1, 0), (-math.inf, -1e38, 1), (NAN, 1, 0)]),
    (synth.EQ, [(1, 1, 1), (1, 2, 0), (0.0, -0.0, 1), (NAN, NAN, 0), (math.inf, math.inf, 1)]),
    (synth.AND, [(0, 0, 0), (0, 5, 0), (3, 0, 0), (2, -7, 1), (-0.0, 1, 0), (NAN, 1, 1), (1e-45, 1, 1)]),
    (synth.OR, [(0, 0, 0), (0, 5, 1), (3, 0, 1), (-0.0, 0.0, 0), (NAN, 0, 1), (0, -1e-45, 1)]),
])
def test_classification_functions_truth_tables(op, cases):
    """Comparisons give 1 or 0 (false whenever a NaN is involved, IEEE);
    AND / OR treat every non-zero value, NaN included, as true."""
    for a, b, want in cases:
        got = oracle.apply(op, a, b)
        assert got == f32(want) and not math.copysign(1.0, got) < 0, (op, a, b, got)


def test_if_selects_on_non_zero():
    for a, want in [(0.0, "c"), (-0.0, "c"), (1.0, "b"), (-2.5, "b"), (NAN, "b"), (1e-45, "b"), (math.inf, "b")]:
        got = oracle.apply3(synth.IF, a, 7.0, -3.0)
        assert got == (f32(7) if want == "b" else f32(-3)), (a, got)
    # the selected operand is returned unchanged, signed zeros and NaN included
    assert math.copysign(1.0, oracle.apply3(synth.IF, 1.0, -0.0, 5.0)) < 0
    assert math.isnan(oracle.apply3(synth.IF, 0.0, 1.0, NAN))


def test_classification_trees_closed_forms():
    """IF over comparisons builds max and |x| (nonzero, distinct inputs, so
    signed zeros and ties do not arise); AND/OR of comparisons build
    interval tests, checked against numpy's float32 comparisons."""
    rng = synth.rng_for(71)
    a = rng.uniform(-5, 5, 2000).astype(np.float32)
    b = rng.uniform(-5, 5, 2000).astype(np.float32)
    keep = (a != b) & (a != 0) & (b != 0)
    X = np.stack([a[keep], b[keep]])
    assert np.array_equal(one("(if (> x0 x1) x0 x1)", X)[0], np.maximum(X[0], X[1]))
    assert np.array_equal(one("(if (< x0 x1) x0 x1)", X)[0], np.minimum(X[0], X[1]))
    assert np.array_equal(one("(if (< x0 0) (- 0 x0) x0)", X)[0], np.abs(X[0]))
    inside = ((X[0] > -1) & (X[0] < 2)).astype(np.float32)
    assert np.array_equal(one("(and (> x0 -1) (< x0 2))", X)[0], inside)
    outside = ((X[0] < -1) | (X[0] > 2)).astype(np.float32)
    assert np.array_equal(one("(or (< x0 -1) (> x0 2))", X)[0], outside)
    # x == x is 1 for every non-NaN x, and IF with equal branches is the branch
    assert np.all(one("(== x0 x0)", X)[0] == 1)
    assert np.array_equal(one("(if x0 x1 x1)", X)[0], X[1])


def test_class_fitness_closed_forms():
    """Decoding is rint (ties to even) and the fitness counts mismatches."""
    rng = synth.rng_for(72)
    X = rng.uniform(-3, 3, (1, 1000)).astype(np.float32)
    y = (X[0] > 0).astype(np.float32)           # class 1 where x0 > 0, else 0
    p = progs.pop("(if (> x0 0) 1 0)", "(if (> x0 0) 0 1)", "(> x0 0)", "0.4", "-0.4", "0.6")
    got = oracle.eval_tree(p.tok, p.cst, p.off, X, y, "class_err")
    n1 = int(y.sum())
    assert got.dtype == np.int32
    assert list(got) == [0, 1000, 0, n1, n1, 1000 - n1]
    ties = progs.pop("2.5", "3.5", "-0.5", "1e30")
    yy = np.array([2.0, 4.0, 0.0, 1e30], np.float32)
    for k in range(4):
        g = oracle.eval_tree(ties.tok, ties.cst, ties.off, X[:, :4], np.full(4, yy[k], np.float32), "class_err")
        assert g[k] == 0, (k, g)
    nan = progs.pop("(/ (- x0 x0) (* 0 x0))", "(log 0)")   # 0 / 0 is protected: 1; log 0 -> 0
    g = oracle.eval_tree(nan.tok, nan.cst, nan.off, X, np.ones(1000, np.float32), "class_err")
    assert list(g) == [0, 1000]


def test_classification_recursive_and_rpn_agree():
    """The recursive interpreter and the one-dimensional-stack RPN
    interpreter evaluate trees with IF to the same bits."""
    rng = synth.rng_for(73)
    pop = synth.ptc2_population(rng, 60, synth.SHUTTLE_SET, 3, 1, 60, 0.25, crange=(-2.0, 2.0))
    X = synth.uniform_cases(rng, 3, 25, -2, 2)
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert np.any((pop.tok & 0xFF) == synth.IF)
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        rt, rc = oracle.prefix_to_rpn(t, c)
        for cc in range(X.shape[1]):
            v, _, _ = oracle.rpn_eval(rt, rc, X, cc)
            assert v.view(np.int32) == ref[p, cc].view(np.int32) or (np.isnan(v) and np.isnan(ref[p, cc]))


def test_register_form_takes_binary_classification_functions_only():
    rng = synth.rng_for(74)
    X = synth.uniform_cases(rng, 2, 50, -2, 2)
    code = np.array([synth.lin_word(synth.GT, 0, 2, 3), synth.lin_word(synth.AND, 0, 0, 1)], np.uint32)
    out = oracle.linear_outputs(code, np.array([0, 2]), np.zeros(0, np.float32), np.array([0, 0]), 2, X)
    # r1 starts as x1: r0 = (x0 > x1) AND x1
    assert np.array_equal(out[0], ((X[0] > X[1]) & (X[1] != 0)).astype(np.float32))
    bad = np.array([synth.lin_word(synth.IF, 0, 2, 3)], np.uint32)
    with pytest.raises(ValueError):
        oracle.linear_outputs(bad, np.array([0, 1]), np.zeros(0, np.float32), np.array([0, 0]), 2, X)
