"""Trees that need many stack levels once lowered (section 5's stack-operand
form with the deeper operand evaluated first).  A binary function whose
operands are both subtrees needs one level more than them when they need the
same; IF evaluates its three operands deepest first and keeps each result on
the stack, so three operands of equal need cost two levels more.  The
smallest tree needing k levels therefore grows like 2^k without IF and like
3^(k/2) with it."""
import numpy as np

import synth


class Tree:
    def __init__(self, rng, n_feat, ops=(synth.ADD, synth.SUB, synth.MUL), crange=(-1.0, 1.0)):
        self.rng, self.n_feat, self.ops, self.crange = rng, n_feat, ops, crange
        self.tok, self.cst = [], []

    def leaf(self):
        if self.rng.random() < 0.6:
            self.tok.append(synth.var_tok(int(self.rng.integers(self.n_feat))))
            self.cst.append(0.0)
        else:
            self.tok.append(synth.CONST)
            self.cst.append(float(np.float32(self.rng.uniform(*self.crange))))

    def fn(self, op):
        self.tok.append(op)
        self.cst.append(0.0)

    def full(self, h):
        """A full binary tree of height h: needs h levels, 2^(h+1) - 1 nodes."""
        if h == 0:
            return self.leaf()
        self.fn(self.ops[int(self.rng.integers(len(self.ops)))])
        self.full(h - 1)
        self.full(h - 1)

    def full_if(self, h):
        """A full IF tree of height h over terminals: needs 2h + 1 levels."""
        if h == 0:
            return self.leaf()
        self.fn(synth.IF)
        for _ in range(3):
            self.full_if(h - 1)

    def pair(self, sub):
        """A binary function of two copies of the shape `sub` builds: one
        level more than `sub` needs."""
        self.fn(self.ops[int(self.rng.integers(len(self.ops)))])
        sub()
        sub()

    def triple(self, sub):
        """IF over three copies of `sub`: two levels more than `sub` needs."""
        self.fn(synth.IF)
        for _ in range(3):
            sub()

    def lists(self):
        return np.array(self.tok, np.int32), np.array(self.cst, np.float32)


def need20(rng, n_feat):
    """IF over three trees of need 18, each a binary function of two full IF
    trees of height 8 (need 17): 59,050 nodes, needing 20 levels, the most
    any tree of at most 65,536 nodes needs."""
    t = Tree(rng, n_feat, ops=(synth.ADD, synth.SUB, synth.MUL, synth.GT, synth.LT))
    t.triple(lambda: t.pair(lambda: t.full_if(8)))
    return t.lists()
