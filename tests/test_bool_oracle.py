"""Pins of the oracle's Boolean (sub-machine-code) evaluator: bit-packed
evaluation against case-by-case evaluation, known solutions of the
multiplexer problem, and closed forms."""
import numpy as np
import pytest

import oracle
import synth
from tests import boolprogs as bp


def test_mux_cases_definition():
    # 6-multiplexer: case c has input f = bit f of c; target = D[address]
    Xw, yw, n = synth.mux_cases(2)
    assert n == 64 and Xw.shape == (6, 2)
    for c in range(n):
        w, b = divmod(c, 32)
        bits = [(Xw[f, w] >> b) & 1 for f in range(6)]
        assert bits == [(c >> f) & 1 for f in range(6)]
        addr = bits[0] + 2 * bits[1]
        assert (yw[w] >> b) & 1 == bits[2 + addr]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_mux_solution_scores_every_case(k):
    Xw, yw, n = synth.mux_cases(k)
    sol = bp.mux_solution(k)
    pop = bp.pop_of(sol)
    assert oracle.eval_bool(pop.tok, pop.off, Xw, n, yw)[0] == n
    # its complement gets none right
    pop2 = bp.pop_of(bp.NOT(list(sol)))
    assert oracle.eval_bool(pop2.tok, pop2.off, Xw, n, yw)[0] == 0


def test_packed_matches_case_by_case():
    # random trees on the 11-multiplexer, every one of the 2048 cases
    Xw, yw, n = synth.mux_cases(3)
    rng = synth.rng_for(61)
    pop = synth.ptc2_population(rng, 40, synth.BOOL_SET, 11, 1, 60, 0.0)
    out = oracle.bool_outputs(pop.tok, pop.off, Xw)
    hits = oracle.eval_bool(pop.tok, pop.off, Xw, n, yw)
    for p in range(pop.n_prog):
        tok, _ = pop.program(p)
        h = 0
        for c in range(n):
            bits = [(c >> f) & 1 for f in range(11)]
            v = bp.eval_case(tok, bits)
            w, b = divmod(c, 32)
            assert bool((out[p, w] >> b) & 1) == v
            target = bits[3 + bits[0] + 2 * bits[1] + 4 * bits[2]]
            h += int(v == bool(target))
        assert hits[p] == h


def test_closed_forms_and_ragged_tail():
    rng = synth.rng_for(62)
    W = 5
    Xw = rng.integers(0, 2**32, size=(3, W), dtype=np.uint64).astype(np.uint32)
    yw = rng.integers(0, 2**32, size=W, dtype=np.uint64).astype(np.uint32)
    x0 = bp.var(0)
    progs = [bp.NOT(x0),                                    # NOT x0
             bp.fn(synth.NOR, x0, x0),                      # NOT x0 again
             bp.fn(synth.AND, x0, bp.NOT(x0)),              # always 0
             bp.fn(synth.OR, x0, bp.NOT(x0)),               # always 1
             x0]
    pop = bp.pop_of(*progs)
    out = oracle.bool_outputs(pop.tok, pop.off, Xw)
    assert (out[0] == ~Xw[0]).all() and (out[1] == ~Xw[0]).all()
    assert (out[2] == 0).all() and (out[3] == 0xFFFFFFFF).all() and (out[4] == Xw[0]).all()
    for n in (1, 31, 33, 100, 160):
        h = oracle.eval_bool(pop.tok, pop.off, Xw, n, yw)
        ybits = np.unpackbits(yw.view(np.uint8), bitorder="little")[:n]
        xbits = np.unpackbits(Xw[0].view(np.uint8), bitorder="little")[:n]
        assert h[2] == int((ybits == 0).sum()) and h[3] == int((ybits == 1).sum())
        assert h[4] == int((xbits == ybits).sum())
        assert h[0] + h[4] == n                             # a program and its complement


def test_rejects_other_functions():
    Xw, yw, n = synth.mux_cases(1)
    for bad in ([synth.ADD] + bp.var(0) + bp.var(1), [synth.CONST], bp.var(7)):
        pop = bp.pop_of(bad)
        with pytest.raises(ValueError):
            oracle.eval_bool(pop.tok, pop.off, Xw, n, yw)
