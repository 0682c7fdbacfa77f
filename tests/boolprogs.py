"""Hand-built Boolean trees for the multiplexer tests (test-side only)."""
import numpy as np

import synth


def var(f):
    return [synth.var_tok(f)]


def fn(op, a, b):
    return [op] + a + b


def NOT(a):
    # NAND(a, a) is NOT a
    return fn(synth.NAND, a, a)


def balanced(op, terms):
    while len(terms) > 1:
        nxt = [fn(op, terms[i], terms[i + 1]) for i in range(0, len(terms) - 1, 2)]
        if len(terms) % 2:
            nxt.append(terms[-1])
        terms = nxt
    return terms[0]


def mux_solution(k):
    """A correct k-address multiplexer: OR over d of (address == d) AND D_d,
    with inputs numbered as in synth.mux_cases (address bits first)."""
    terms = []
    for d in range(1 << k):
        lits = [var(i) if (d >> i) & 1 else NOT(var(i)) for i in range(k)]
        terms.append(fn(synth.AND, balanced(synth.AND, lits), var(k + d)))
    return np.asarray(balanced(synth.OR, terms), np.int32)


def pop_of(*toks):
    return synth.trees_from_lists([(np.asarray(t, np.int32), np.zeros(len(t), np.float32)) for t in toks])


def eval_case(tok, bits):
    """Value of a prefix Boolean tree on one case given its input bits
    (Python bools, one case at a time)."""
    pos = 0

    def rd():
        nonlocal pos
        t = int(tok[pos])
        pos += 1
        op = t & 0xFF
        if op == synth.VAR:
            return bool(bits[t >> 8])
        a, b = rd(), rd()
        if op == synth.AND:
            return a and b
        if op == synth.OR:
            return a or b
        if op == synth.NAND:
            return not (a and b)
        return not (a or b)

    v = rd()
    assert pos == len(tok)
    return v
