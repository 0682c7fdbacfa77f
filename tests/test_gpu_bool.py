"""GPU parity of the Boolean (sub-machine-code) kernels against the oracle:
output words and hit counts are integers, so the bar is bit-exact."""
import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests import boolprogs as bp
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def dev_u32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")


def gpu_bool(pop, Xw, yw, kind, n_cases):
    import torch
    P, W = pop.n_prog, Xw.shape[1]
    out = torch.empty((P, W) if kind == "cases" else P, dtype=torch.int32, device="cuda")
    gp.gp_eval_bool(pop.tok, pop.off, dev_u32(Xw), dev_u32(yw) if yw is not None else None, kind, out, n_cases)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    return r.view(np.uint32) if kind == "cases" else r


@pytest.mark.parametrize("F,W,n_cases,depth_hi", [
    (20, 3000, 3000 * 32 - 5, 120),     # 20 inputs: the 8-slot kernel; ragged last word
    (32, 1500, 1500 * 32, 120),         # 32 inputs: the 4-slot kernel
    (6, 777, 777 * 32 - 31, 300),       # deep trees
    (3, 1, 1, 40),                      # one case
])
def test_bool_words_and_hits_match_oracle(F, W, n_cases, depth_hi):
    rng = synth.rng_for(700 + F)
    pop = synth.ptc2_population(rng, 150, synth.BOOL_SET, F, 1, depth_hi, 0.0)
    Xw = rng.integers(0, 2**32, size=(F, W), dtype=np.uint64).astype(np.uint32)
    yw = rng.integers(0, 2**32, size=W, dtype=np.uint64).astype(np.uint32)
    say("bool F=%d W=%d n=%d: words" % (F, W, n_cases))
    got = gpu_bool(pop, Xw, None, "cases", n_cases)
    ref = oracle.bool_outputs(pop.tok, pop.off, Xw)
    assert (got == ref).all()
    say("bool F=%d W=%d n=%d: hits" % (F, W, n_cases))
    hits = gpu_bool(pop, Xw, yw, "hits", n_cases)
    assert (hits == oracle.eval_bool(pop.tok, pop.off, Xw, n_cases, yw)).all()


def test_mux20_full_size_solution_and_sample():
    """The 20-multiplexer over all 2^20 cases: a correct program scores every
    case, its complement none, and sampled random programs match the oracle."""
    Xw, yw, n = synth.mux_cases(4)
    w = synth.mux_workload()
    sol = bp.mux_solution(4)
    idx = np.linspace(0, w.pop.n_prog - 1, 24).astype(int)
    sample = [w.pop.program(int(i))[0] for i in idx]
    pop = bp.pop_of(sol, bp.NOT(list(sol)), *sample)
    say("mux20: solution and sample")
    hits = gpu_bool(pop, Xw, yw, "hits", n)
    assert hits[0] == n and hits[1] == 0
    assert (hits == oracle.eval_bool(pop.tok, pop.off, Xw, n, yw)).all()
    # the whole benchmark population through a resident set, in the bench's launch shape
    import torch
    say("mux20: resident set of the benchmark population")
    ps = gp.ProgSet.boolean(w.pop.tok, w.pop.off, Xw.shape[0])
    out = torch.empty(w.pop.n_prog, dtype=torch.int32, device="cuda")
    ps.eval(dev_u32(Xw), dev_u32(yw), "hits", out, n_cases=n)
    torch.cuda.synchronize()
    allh = out.cpu().numpy()
    ps.close()
    assert (allh[idx] == hits[2:]).all()
    assert (allh >= 0).all() and (allh <= n).all()


def test_bool_rejects():
    import torch
    Xw = dev_u32(np.zeros((2, 4), np.uint32))
    out = torch.empty(1, dtype=torch.int32, device="cuda")
    add = bp.pop_of([synth.ADD] + bp.var(0) + bp.var(1))
    with pytest.raises(gp.GPError) as e:
        gp.gp_eval_bool(add.tok, add.off, Xw, Xw[0], "hits", out, 128)
    assert e.value.status == gp.GP_E_INVAL
    ok = bp.pop_of(bp.fn(synth.AND, bp.var(0), bp.var(1)))
    with pytest.raises(gp.GPError):
        gp.gp_eval_bool(ok.tok, ok.off, Xw, Xw[0], "mse", out, 128)
    # the arithmetic entry points reject the bitwise-only functions (AND and OR are
    # logical there, a classification function)
    nand = bp.pop_of(bp.fn(synth.NAND, bp.var(0), bp.var(1)))
    with pytest.raises(gp.GPError):
        gp.gp_eval_tree(nand.tok, np.zeros(3, np.float32), nand.off, torch.zeros((2, 8), device="cuda"), None,
                        "cases", torch.empty((1, 8), device="cuda"))
