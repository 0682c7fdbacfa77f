"""Programs deeper than the fast kernels hold (more than 12 stack levels) run
on the deep kernel variants and match the oracle bit for bit; with more than
32 features read, 12 levels is the limit and deeper programs are refused."""
import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests import deeptrees
from tests.gpu_util import dev, fitness_close, gpu_tree, same_bits, say

pytestmark = pytest.mark.gpu


def _cases(rng, n_feat, n):
    # small integers (many zeros, so IF takes both branches) and reals
    X = rng.uniform(-2, 2, (n_feat, n)).astype(np.float32)
    X[:, ::3] = np.round(X[:, ::3])
    return X


def _check(pop, X):
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert same_bits(got, ref).all()
    y = np.asarray(ref[0], np.float32) * np.float32(0.5)
    y = np.where(np.isfinite(y), y, np.float32(0))
    fit = gpu_tree(pop, X, y, "sum_abs")
    assert fitness_close(fit, oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, "sum_abs")).all()


def test_full_binary_tree_of_height_15():
    """65,535 nodes needing 15 levels: the deepest binary tree within the
    length limit."""
    rng = synth.rng_for(900)
    t = deeptrees.Tree(rng, 3, crange=(-1.2, 1.2))
    t.full(15)
    pop = synth.trees_from_lists([t.lists()])
    say("full binary tree, 15 levels")
    _check(pop, _cases(rng, 3, 333))


def test_if_tree_needing_20_levels():
    rng = synth.rng_for(901)
    pop = synth.trees_from_lists([deeptrees.need20(rng, 4)])
    say("IF tree, 20 levels")
    _check(pop, _cases(rng, 4, 321))


def test_population_with_one_deep_program():
    """One program of 14 levels moves the whole set to a deep kernel; every
    program still matches the oracle."""
    rng = synth.rng_for(902)
    pop = synth.ptc2_population(rng, 300, synth.SHUTTLE_SET, 9, 1, 200, 0.1, crange=(-3.0, 3.0))
    t = deeptrees.Tree(rng, 9, ops=(synth.ADD, synth.MUL, synth.PDIV, synth.GT))
    t.pair(lambda: t.full_if(6))                 # 13 + 1 levels
    progs = [pop.program(i) for i in range(pop.n_prog)]
    progs.insert(150, t.lists())
    both = synth.trees_from_lists(progs)
    _, st = gp.gp_lower_tree(*t.lists(), 9)
    assert st["max_depth"] == 14
    say("300 trees + one of 14 levels")
    _check(both, _cases(rng, 9, 1000))
    ps = gp.ProgSet.tree(both.tok, both.cst, both.off, 9)
    assert ps.info()["max_depth"] == 14


def test_deep_programs_with_transcendentals():
    rng = synth.rng_for(903)
    t = deeptrees.Tree(rng, 2, ops=(synth.ADD, synth.SUB, synth.MUL, synth.PDIV))
    t.full(13)
    tok, cst = t.lists()
    # one sin/cos/exp/log above the deep part; transcendentals are within 2 ulp per
    # operation, so only the cases where the deep part is bit-exact are compared bit for bit
    pop = synth.trees_from_lists([(np.concatenate([[op], tok]), np.concatenate([[0.0], cst]).astype(np.float32))
                                  for op in (synth.SIN, synth.COS, synth.EXPC, synth.PLOG)] + [(tok, cst)])
    X = _cases(rng, 2, 500)
    say("deep trees under sin/cos/exp/log")
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert same_bits(got[4], ref[4]).all()
    from tests.gpu_util import ulp_dist, ULP_TRANSC
    fin = np.isfinite(ref[4])
    assert (ulp_dist(got[:4][:, fin], ref[:4][:, fin]) <= ULP_TRANSC).all()


def test_wide_programs_up_to_twelve_levels():
    """41 features: 12 levels run (the KDD-width deep kernel); 13 are refused
    with GP_E_DEPTH."""
    rng = synth.rng_for(904)
    t = deeptrees.Tree(rng, 41, ops=(synth.ADD, synth.MUL, synth.LT, synth.PDIV))
    t.fn(synth.SIN)                              # one exit to the binary64 code at the root
    t.pair(lambda: t.full_if(5))                 # 11 + 1 levels
    pop = synth.trees_from_lists([t.lists()])
    X = _cases(rng, 41, 700)
    say("41 features, 12 levels")
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    from tests.gpu_util import ulp_dist
    assert (same_bits(got, ref) | (ulp_dist(got, ref) <= 2)).all()
    t = deeptrees.Tree(rng, 41)
    t.full_if(6)                                 # 13 levels
    pop = synth.trees_from_lists([t.lists()])
    say("41 features, 13 levels: refused")
    with pytest.raises(gp.GPError) as e:
        gpu_tree(pop, X, None, "cases")
    assert e.value.status == gp.GP_E_DEPTH


def test_deep_boolean_tree():
    """A full Boolean tree of height 14 (32,767 nodes) on packed cases."""
    import torch
    rng = synth.rng_for(905)
    t = deeptrees.Tree(rng, 6, ops=synth.BOOL_SET)
    t.full(14)
    tok = np.array([x if x != synth.CONST else synth.var_tok(0) for x in t.tok], np.int32)
    off = np.array([0, len(tok)], np.int64)
    W = 300
    Xw = rng.integers(0, 2**32, size=(6, W), dtype=np.uint64).astype(np.uint32)
    yw = rng.integers(0, 2**32, size=W, dtype=np.uint64).astype(np.uint32)
    out = torch.empty((1, W), dtype=torch.int32, device="cuda")
    Xd = dev(Xw.view(np.int32))
    say("Boolean tree, 14 levels")
    gp.gp_eval_bool(tok, off, Xd, None, "cases", out, W * 32)
    torch.cuda.synchronize()
    assert (out.cpu().numpy().view(np.uint32) == oracle.bool_outputs(tok, off, Xw)).all()
    hits = torch.empty(1, dtype=torch.int32, device="cuda")
    gp.gp_eval_bool(tok, off, Xd, dev(yw.view(np.int32)), "hits", hits, W * 32 - 7)
    torch.cuda.synchronize()
    assert hits.cpu().numpy()[0] == oracle.eval_bool(tok, off, Xw, W * 32 - 7, yw)[0]
