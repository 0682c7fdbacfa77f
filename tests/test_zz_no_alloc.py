"""gp_progset_eval_noalloc: the program-set evaluation with nothing allocated
during the call, against gp_progset_eval on the same inputs (bit for bit),
on two calls in a row, the second with fewer cases; and its size limit."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests.gpu_util import fitness_close, say

pytestmark = pytest.mark.gpu


def _data(rng, F, n):
    import torch
    X = synth.uniform_cases(rng, F, n, -3, 3)
    y = synth.gaussian_noise(rng, n, 1.0)
    return X, y, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()


def test_noalloc_matches_progset_eval_twice():
    import torch
    rng = synth.rng_for(91)
    pop = synth.ptc2_population(rng, 700, synth.FULL, 6, 1, 200, 1 / 7)
    ps = gp.ProgSet.tree(pop.tok, pop.cst, pop.off, 6)
    for n, kind in ((70001, "mse"), (3001, "sum_abs")):
        X, y, Xd, yd = _data(rng, 6, n)
        say("no-alloc vs progset, %d cases, %s" % (n, kind))
        a = gp.out_tensor(kind, pop.n_prog, n)
        b = gp.out_tensor(kind, pop.n_prog, n)
        a.fill_(-3)
        b.fill_(-4)
        ps.eval(Xd, yd, kind, a)
        ps.eval_noalloc(Xd, yd, kind, b)
        torch.cuda.synchronize()
        ga, gb = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(ga.view(np.int32), gb.view(np.int32))
        ref = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, kind, threads=8)
        assert fitness_close(gb, ref).mean() >= 0.98
    ps.close()


def test_noalloc_linear_hits_and_cases():
    import torch
    rng = synth.rng_for(92)
    lp = synth.linear_population(rng, 300, 8, 120, synth.BASIC, 8, 16, n_const=2)
    ps = gp.ProgSet.linear(lp.code, lp.off, lp.cst, lp.cst_off, lp.n_reg, 16)
    for n in (40000, 513):
        X = synth.normal_cases(rng, 16, n)
        _, y = synth.sign_labels(rng, X)
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        say("no-alloc linear hits, %d cases" % n)
        h = gp.out_tensor("hits", lp.n_prog, n)
        ps.eval_noalloc(Xd, yd, "hits", h)
        c = gp.out_tensor("cases", lp.n_prog, n)
        ps.eval_noalloc(Xd, yd, "cases", c)
        torch.cuda.synchronize()
        ref = oracle.eval_linear(lp.code, lp.off, lp.cst, lp.cst_off, lp.n_reg, X, y, "hits", threads=8)
        assert np.array_equal(h.cpu().numpy(), ref)
        refc = oracle.linear_outputs(lp.code, lp.off, lp.cst, lp.cst_off, lp.n_reg, X)
        assert np.array_equal(c.cpu().numpy().view(np.int32), refc.view(np.int32))
    ps.close()


def test_noalloc_rejects_more_partials_than_it_holds():
    import torch
    rng = synth.rng_for(93)
    pop = synth.ptc2_population(rng, 2100, synth.BASIC, 2, 1, 20, 0.3)
    ps = gp.ProgSet.tree(pop.tok, pop.cst, pop.off, 2)
    n = 256 * 1000                     # 2100 x 1000 blocks > 2^21 partial sums
    X, y, Xd, yd = _data(rng, 2, n)
    out = gp.out_tensor("mse", pop.n_prog, n)
    with pytest.raises(gp.GPError) as e:
        ps.eval_noalloc(Xd, yd, "mse", out)
    assert e.value.status == gp.GP_E_NOMEM
    # a smaller call still works afterwards
    n = 256 * 900
    X, y, Xd, yd = _data(rng, 2, n)
    a = gp.out_tensor("mse", pop.n_prog, n)
    b = gp.out_tensor("mse", pop.n_prog, n)
    ps.eval(Xd, yd, "mse", a)
    ps.eval_noalloc(Xd, yd, "mse", b)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    ps.close()
