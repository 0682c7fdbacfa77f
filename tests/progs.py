"""Small helpers for writing test programs by hand (test-side only)."""
import numpy as np

import synth

_OPS = {"+": synth.ADD, "-": synth.SUB, "*": synth.MUL, "/": synth.PDIV,
        "sin": synth.SIN, "cos": synth.COS, "exp": synth.EXPC, "log": synth.PLOG,
        ">": synth.GT, "<": synth.LT, "==": synth.EQ, "and": synth.AND, "or": synth.OR, "if": synth.IF}


def _lex(s):
    return s.replace("(", " ( ").replace(")", " ) ").split()


def parse(s):
    """Parse an s-expression like "(+ (* x0 x0) 0.5)" into prefix arrays."""
    toks = _lex(s)
    out_t, out_c = [], []
    pos = 0

    def rd():
        nonlocal pos
        t = toks[pos]
        pos += 1
        if t == "(":
            op = toks[pos]
            pos += 1
            out_t.append(_OPS[op]); out_c.append(0.0)
            n = 0
            while toks[pos] != ")":
                rd()
                n += 1
            pos += 1
            assert n == synth.ARITY[_OPS[op]], s
        elif t[0] == "x":
            out_t.append(synth.var_tok(int(t[1:]))); out_c.append(0.0)
        else:
            out_t.append(synth.CONST); out_c.append(np.float32(float(t)))

    rd()
    assert pos == len(toks)
    return np.asarray(out_t, np.int32), np.asarray(out_c, np.float32)


def pop(*exprs):
    return synth.trees_from_lists([parse(e) for e in exprs])


def tree_to_register_lgp(tok, cst, n_reg):
    """Translate one prefix tree into an equivalent register program: each
    function writes the register named by its stack height (post-order,
    left operand first), terminals are read directly as feature ids or
    constants.  Returns (code, consts) or None if it needs more than n_reg
    registers or more than 128 constants."""
    tok = [int(t) for t in tok]
    consts = []
    code = []

    def walk(i, h):
        # returns (next index, source id of the value)
        op = tok[i] & 0xFF
        if op == synth.VAR:
            return i + 1, n_reg + (tok[i] >> 8)
        if op == synth.CONST:
            consts.append(np.float32(cst[i]))
            return i + 1, 128 + len(consts) - 1
        if synth.ARITY[op] == 1:
            j, a = walk(i + 1, h)
            if h >= n_reg:
                raise OverflowError
            code.append(synth.lin_word(op, h, a, 0))
            return j, h
        j, a = walk(i + 1, h)
        # if the left value sits in register h, the right subtree must not clobber it
        hb = h + 1 if a == h else h
        k, b = walk(j, hb)
        if h >= n_reg:
            raise OverflowError
        code.append(synth.lin_word(op, h, a, b))
        return k, h

    try:
        _, src = walk(0, 0)
    except OverflowError:
        return None
    if src != 0:
        # lone terminal: copy it into r0 with x + 0 would change -0; use a
        # multiply-free identity instead: r0 = src - 0 keeps every value except
        # NaN payloads, so only trees with a function at the root are used.
        return None
    if len(consts) > 128:
        return None
    return np.asarray(code, np.uint32), np.asarray(consts, np.float32)
