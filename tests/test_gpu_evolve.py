"""Whole GP runs on the GPU (gp_evolve): reproducible from the seed, the
best-so-far fitness never gets worse, and the reported best fitness is what
the evaluator and the oracle give for the reported best program."""
import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests.gpu_util import dev, fitness_close, say

pytestmark = pytest.mark.gpu

SEXTIC_SET = (synth.MUL, synth.PDIV, synth.ADD, synth.SUB, synth.SIN, synth.COS, synth.PLOG, synth.EXPC)


def sextic(n, seed):
    rng = synth.rng_for(seed)
    x = rng.uniform(-1, 1, n)
    y = (x ** 6 - 2 * x ** 4 + x ** 2).astype(np.float32)
    return x.astype(np.float32)[None, :], y


def test_sextic_run():
    import torch
    X, y = sextic(5000, 81)
    Xd, yd = dev(X), dev(y)
    cfg = gp.evolve_config(SEXTIC_SET, kind="mse", pop_size=200, generations=6, seed=3)
    say("sextic run 1")
    r1 = gp.evolve(cfg, Xd, yd)
    say("sextic run 2")
    r2 = gp.evolve(cfg, Xd, yd)
    assert r1["best_fitness"] == r2["best_fitness"]
    assert np.array_equal(r1["best_tok"], r2["best_tok"])
    b = r1["best_per_generation"]
    assert len(b) == 7 and (np.diff(b) <= 0).all()
    assert r1["gp_ops"] % 5000 == 0 and r1["gp_ops"] >= 200 * 7 * 5000
    # the best program alone: the same fitness bits from the evaluator, and the oracle's within tolerance
    tok, cst = r1["best_tok"], r1["best_cst"]
    off = np.array([0, len(tok)], np.int64)
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    gp.gp_eval_tree(tok, cst, off, Xd, yd, "mse", out)
    torch.cuda.synchronize()
    alone = float(out.cpu().numpy()[0])
    assert np.float32(r1["best_fitness"]) == np.float32(alone)
    ref = oracle.eval_tree(tok, cst, off, X, y, "mse")
    assert fitness_close(np.array([alone], np.float32), ref).all(), (alone, ref)


def test_boolean_run():
    import torch
    Xw, yw, n = synth.mux_cases(3)          # the 11-multiplexer, 2048 cases
    Xd = torch.from_numpy(Xw.view(np.int32)).cuda()
    yd = torch.from_numpy(yw.view(np.int32)).cuda()
    cfg = gp.evolve_config(synth.BOOL_SET, kind="hits", pop_size=300, generations=8, seed=5)
    say("11-multiplexer run")
    r = gp.evolve(cfg, Xd, yd, n_cases=n)
    b = r["best_per_generation"]
    assert (np.diff(b) >= 0).all() and 0 < b[-1] <= n
    tok = r["best_tok"]
    off = np.array([0, len(tok)], np.int64)
    assert oracle.eval_bool(tok, off, Xw, n, yw)[0] == r["best_fitness"]
