"""The GP run's host steps (gp_init_population, gp_breed) on the CPU:
offspring are well-formed trees of the run's function set within the size
and depth limits, runs are reproducible from their seed, and tournament
selection favours better scores."""
import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth

ARITH = (synth.ADD, synth.SUB, synth.MUL, synth.PDIV, synth.SIN, synth.COS, synth.EXPC, synth.PLOG)


def arity(t):
    op = t & 0xFF
    if op in (synth.VAR, synth.CONST):
        return 0
    return synth.ARITY[op]


def depth(tok):
    """edges on the longest root-to-leaf path, by recursion over the prefix form"""
    pos = 0

    def rd():
        nonlocal pos
        a = arity(int(tok[pos]))
        pos += 1
        return 0 if a == 0 else 1 + max(rd() for _ in range(a))

    d = rd()
    assert pos == len(tok)
    return d


def check_population(tok, cst, off, cfg, n_feat, fset):
    assert len(off) == cfg.pop_size + 1 and off[0] == 0
    X = synth.uniform_cases(synth.rng_for(1), n_feat, 3, -1, 1)
    # the oracle accepts every program (well-formed, features in range)
    if set(fset) <= set(synth.BOOL_SET):
        Xw = np.zeros((n_feat, 1), np.uint32)
        oracle.bool_outputs(tok, off, Xw)
    else:
        oracle.tree_outputs(tok, cst, off, X)
    for p in range(cfg.pop_size):
        t = tok[off[p]:off[p + 1]]
        assert 1 <= len(t) <= cfg.max_size
        assert depth(t) <= cfg.max_depth
        ops = {int(x) & 0xFF for x in t if arity(int(x)) > 0}
        assert ops <= set(fset)


def test_init_population_ramped_and_valid():
    cfg = gp.evolve_config(ARITH, pop_size=200, p_const=0.3, seed=5)
    tok, cst, off = gp.init_population(cfg, 3)
    check_population(tok, cst, off, cfg, 3, ARITH)
    depths = [depth(tok[off[p]:off[p + 1]]) for p in range(200)]
    # full trees (odd positions) reach their ramp depth 2 .. 6 exactly
    for p in range(1, 200, 2):
        assert depths[p] == 2 + (p // 2) % 5
    assert max(depths) <= 6
    # constants appear, within the range
    c = cst[(tok & 0xFF) == synth.CONST]
    assert len(c) > 0 and (c >= -1).all() and (c < 1).all()


def test_reproducible_from_seed():
    cfg = gp.evolve_config(ARITH, pop_size=64, seed=9)
    a = gp.init_population(cfg, 2)
    b = gp.init_population(cfg, 2)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    score = np.arange(64, dtype=np.float64)
    n1 = gp.breed(cfg, *a, 2, score, 77)
    n2 = gp.breed(cfg, *a, 2, score, 77)
    n3 = gp.breed(cfg, *a, 2, score, 78)
    assert all(np.array_equal(x, y) for x, y in zip(n1, n2))
    assert not np.array_equal(n1[0], n3[0])


@pytest.mark.parametrize("max_size,max_depth", [(1000, 50), (25, 50), (1000, 4)])
def test_breed_respects_limits(max_size, max_depth):
    cfg = gp.evolve_config(ARITH, pop_size=150, max_size=max_size, max_depth=max_depth, init_depth=(1, 4),
                           p_const=0.2, seed=3)
    tok, cst, off = gp.init_population(cfg, 4)
    rng = np.random.default_rng(0)
    for g in range(6):
        score = rng.standard_normal(cfg.pop_size)
        tok, cst, off = gp.breed(cfg, tok, cst, off, 4, score, 100 + g)
        check_population(tok, cst, off, cfg, 4, ARITH)


def test_selection_pressure_and_copies():
    # no crossover or mutation: every child is a copy of a tournament winner
    cfg = gp.evolve_config(ARITH, pop_size=300, p_crossover=0.0, p_mutation=0.0, seed=11)
    tok, cst, off = gp.init_population(cfg, 2)
    progs = [tuple(tok[off[p]:off[p + 1]]) for p in range(300)]
    score = np.arange(300, dtype=np.float64)          # program p has score p
    ntok, ncst, noff = gp.breed(cfg, tok, cst, off, 2, score, 5)
    kids = [tuple(ntok[noff[p]:noff[p + 1]]) for p in range(300)]
    assert all(k in set(progs) for k in kids)
    # winners of 7 draws: the mean rank of the minimum of 7 uniform draws is about P / 8
    rank = np.array([min(i for i, q in enumerate(progs) if q == k) for k in kids])
    assert rank.mean() < 300 / 4
    # NaN scores lose every tournament they meet a number in
    score2 = np.full(300, np.nan)
    score2[17] = 1.0
    cfg2 = gp.evolve_config(ARITH, pop_size=300, p_crossover=0.0, p_mutation=0.0, tournament=300, seed=2)
    ntok, ncst, noff = gp.breed(cfg2, tok, cst, off, 2, score2, 6)
    kids = [tuple(ntok[noff[p]:noff[p + 1]]) for p in range(300)]
    # a tournament of 300 draws (with replacement) contains program 17 with
    # probability 1 - (299/300)^300; every such tournament picks it
    p17 = 1 - (299 / 300) ** 300
    n17 = sum(k == progs[17] for k in kids)
    sd = (300 * p17 * (1 - p17)) ** 0.5
    assert abs(n17 - 300 * p17) < 5 * sd, (n17, 300 * p17)


def test_crossover_and_mutation_change_programs():
    cfg = gp.evolve_config(ARITH, pop_size=100, p_crossover=1.0, p_mutation=1.0, seed=4)
    tok, cst, off = gp.init_population(cfg, 3)
    parents = {tuple(tok[off[p]:off[p + 1]]) for p in range(100)}
    ntok, ncst, noff = gp.breed(cfg, tok, cst, off, 3, np.zeros(100), 8)
    kids = [tuple(ntok[noff[p]:noff[p + 1]]) for p in range(100)]
    assert sum(k not in parents for k in kids) > 50


def test_boolean_runs():
    cfg = gp.evolve_config(synth.BOOL_SET, kind="hits", pop_size=80, seed=7)
    tok, cst, off = gp.init_population(cfg, 6)
    check_population(tok, cst, off, cfg, 6, synth.BOOL_SET)
    assert ((tok & 0xFF) != synth.CONST).all()
    tok, cst, off = gp.breed(cfg, tok, None, off, 6, np.zeros(80), 1)
    check_population(tok, cst, off, cfg, 6, synth.BOOL_SET)


def test_classification_runs():
    """The classification set (three-operand IF, logical AND and OR): the
    host steps keep every program well formed and lowerable, and class
    errors are a minimised fitness."""
    cfg = gp.evolve_config(synth.SHUTTLE_SET, kind="class_err", pop_size=120, p_const=0.1,
                           const_range=(-200.0, 200.0), seed=21)
    tok, cst, off = gp.init_population(cfg, 9)
    check_population(tok, cst, off, cfg, 9, synth.SHUTTLE_SET)
    assert np.any((tok & 0xFF) == synth.IF)
    score = np.arange(120, dtype=np.float64)
    nt, nc, no = gp.breed(cfg, tok, cst, off, 9, score, 5)
    check_population(nt, nc, no, cfg, 9, synth.SHUTTLE_SET)
    for p in range(0, 120, 7):
        gp.gp_lower_tree(nt[no[p]:no[p + 1]], nc[no[p]:no[p + 1]], 9)
    # NAND cannot join an arithmetic set
    with pytest.raises(gp.GPError):
        gp.init_population(gp.evolve_config(synth.SHUTTLE_SET + (synth.NAND,), kind="class_err"), 9)


def test_config_errors():
    bad = [gp.evolve_config(ARITH + synth.BOOL_SET),                 # mixed sets
           gp.evolve_config(synth.BOOL_SET, kind="mse"),             # Boolean with an error measure
           gp.evolve_config(()),                                     # empty set
           gp.evolve_config(ARITH, p_crossover=1.5),
           gp.evolve_config(ARITH, init_depth=(5, 2))]
    for cfg in bad:
        with pytest.raises(gp.GPError) as e:
            gp.init_population(cfg, 2)
        assert e.value.status == gp.GP_E_INVAL
    cfg = gp.evolve_config(ARITH, pop_size=10, max_size=1000)
    tok, cst, off = gp.init_population(cfg, 2)
    with pytest.raises(gp.GPError):                                  # a parent with a foreign opcode
        t2 = tok.copy()
        t2[0] = synth.NAND
        gp.breed(cfg, t2, cst, off, 2, np.zeros(10), 1)
