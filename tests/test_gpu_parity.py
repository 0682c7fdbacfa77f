"""GPU parity: the HIP evaluator against the CPU oracle, element by element.

Bar (from the stated contract): per-case outputs bit-exact for + - * and
protected division; within 2 ulp per sin/cos/exp/log operation; fitness sums
within 1e-5 relative; hit counts bit-exact.

Both sides evaluate sin/cos/exp/log in binary64 and round once, so their
results coincide except in rare near-tie cases; the tests check that
per-case outputs of whole programs are identical for almost every case.  A
program may miss the fitness tolerance only if it is ill-conditioned: moving
every transcendental result by 2 ulp moves its oracle fitness by more than
the tolerance (a program no 2-ulp evaluator can reproduce); such misses are
counted and bounded."""
import numpy as np
import pytest

import oracle
import paper_1601_00221_amd as gp
import synth
from tests import progs
from tests.gpu_util import (ULP_TRANSC, fitness_close, gpu_linear, gpu_tree, has_transcendental_tree,
                            same_bits, say, ulp_dist, well_conditioned_tree)

pytestmark = pytest.mark.gpu


def test_device_is_mi355x():
    import torch
    assert torch.cuda.is_available()
    name = torch.cuda.get_device_properties(0).gcnArchName
    say("device arch", name)
    assert name.startswith("gfx950")


# --------------------------------------------------------------------------
# Tiny tree workload (100 ramped half-and-half trees, 1024 cases, sum |e|)
# --------------------------------------------------------------------------
def test_tiny_tree_workload_exact():
    w = synth.tiny_tree_workload()
    y = oracle.tree_outputs(w.target.tok, w.target.cst, w.target.off, w.X)[0]
    say("tiny-tree: cases")
    got_cases = gpu_tree(w.pop, w.X, None, "cases")
    ref_cases = oracle.tree_outputs(w.pop.tok, w.pop.cst, w.pop.off, w.X)
    assert same_bits(got_cases, ref_cases).all()
    say("tiny-tree: sum_abs")
    got = gpu_tree(w.pop, w.X, y, "sum_abs")
    ref = oracle.eval_tree(w.pop.tok, w.pop.cst, w.pop.off, w.X, y, "sum_abs")
    assert fitness_close(got, ref).all()
    # {+,-,*,/p} only: the per-case terms are identical, so the sums agree
    # to the last bit except for the summation order
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) < 1e-6


# --------------------------------------------------------------------------
# Per-operation sweeps
# --------------------------------------------------------------------------
def _sweep_inputs(n=40000, seed=3):
    rng = synth.rng_for(seed)
    special = np.array([0.0, -0.0, 1e-45, -1e-45, 1e-40, 1.17549435e-38, 1e-7, 9.99999997e-7, 1e-6,
                        1.0000001e-6, 0.5, 1.0, -1.0, 2.0, np.pi, -np.pi, 87.9, 88.0, 88.1, 89.0, 100.0,
                        1e4, -1e4, 1e20, -1e20, 3.4e38, -3.4e38, np.inf, -np.inf, np.nan], np.float32)
    r = np.concatenate([
        rng.uniform(-10, 10, n // 4),
        rng.standard_normal(n // 4) * 1e3,
        10.0 ** rng.uniform(-40, 38, n // 4) * rng.choice([-1, 1], n // 4),
        rng.uniform(-100, 100, n // 4),
    ]).astype(np.float32)
    return np.concatenate([special, r]).astype(np.float32)


@pytest.mark.parametrize("expr,bound", [
    ("(sin x0)", ULP_TRANSC), ("(cos x0)", ULP_TRANSC), ("(exp x0)", ULP_TRANSC), ("(log x0)", ULP_TRANSC),
    ("(+ x0 x1)", 0), ("(- x0 x1)", 0), ("(* x0 x1)", 0), ("(/ x0 x1)", 0),
    ("(- x1 x0)", 0), ("(/ x1 x0)", 0), ("(/ x0 1e-6)", 0), ("(/ 3 x1)", 0),
])
def test_single_operation_sweep(expr, bound):
    a = _sweep_inputs()
    b = np.roll(_sweep_inputs(seed=4), 7)
    X = np.stack([a, b])
    pop = progs.pop(expr)
    say("sweep", expr)
    got = gpu_tree(pop, X, None, "cases")[0]
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)[0]
    d = ulp_dist(got, ref)
    i = int(d.argmax())
    assert d.max() <= bound, (expr, X[:, i], got[i], ref[i], int(d.max()))
    assert (np.isnan(got) == np.isnan(ref)).all()
    say("exact: %d of %d" % ((d == 0).sum(), d.size))
    assert (d == 0).mean() >= 0.9999


# --------------------------------------------------------------------------
# Scale-shaped trees at a reduced size: several tiles and a ragged tail
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_feat,n_cases", [(8, 3001), (1, 777), (16, 1500), (32, 600), (9, 64), (3, 65)])
def test_trees_reduced(n_feat, n_cases):
    rng = synth.rng_for(100 + n_feat)
    pop = synth.ptc2_population(rng, 160, synth.FULL, n_feat, 1, 200, 1.0 / (n_feat + 1))
    X = synth.uniform_cases(rng, n_feat, n_cases, -5, 5)
    y = synth.gaussian_noise(rng, n_cases, 1.0)
    say("trees F=%d N=%d: cases" % (n_feat, n_cases))
    got_cases = gpu_tree(pop, X, None, "cases")
    ref_cases = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    tr = has_transcendental_tree(pop)
    assert same_bits(got_cases[~tr], ref_cases[~tr]).all()
    same = same_bits(got_cases, ref_cases)
    say("cases differing: %d of %d" % ((~same).sum(), same.size))
    assert same.mean() >= 0.9999
    for kind in ("mse", "sum_abs"):
        say("trees F=%d N=%d: %s" % (n_feat, n_cases, kind))
        got = gpu_tree(pop, X, y, kind)
        ref, ok = well_conditioned_tree(pop, X, y, kind)
        close = fitness_close(got, ref)
        assert close[~tr].all()
        miss = ~close
        say("programs %d, ill-conditioned %d, fitness misses %d" % (len(got), (~ok).sum(), miss.sum()))
        assert not (miss & ok).any(), (np.nonzero(miss & ok)[0], got[miss & ok], ref[miss & ok])
        assert miss.sum() <= 0.02 * len(got)


def test_arith_trees_bit_exact_cases():
    rng = synth.rng_for(7)
    pop = synth.ptc2_population(rng, 200, synth.ARITH3, 8, 1, 256, 1 / 9)
    X = synth.uniform_cases(rng, 8, 2500, -5, 5)
    say("arith trees: cases")
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert same_bits(got, ref).all()


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------
def test_edge_shapes():
    X = synth.uniform_cases(synth.rng_for(9), 2, 1, -1, 1)
    pop = progs.pop("x0", "1.5", "(+ x0 x1)", "(sin 2)", "(/ 2 0)", "(* (+ x1 x0) (- x0 x1))")
    for n in (1, 63, 64, 65, 511, 512, 513):
        Xn = synth.uniform_cases(synth.rng_for(n), 2, n, -2, 2)
        say("edge N=%d" % n)
        got = gpu_tree(pop, Xn, None, "cases")
        ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, Xn)
        d = ulp_dist(got, ref)
        assert d[[0, 1, 2, 4, 5]].max() == 0 and d[3].max() <= ULP_TRANSC
    y = np.zeros(1, np.float32)
    got = gpu_tree(progs.pop("(+ x0 x1)"), X, y, "sum_abs")
    assert got[0] == np.float32(abs(np.float32(X[0, 0] + X[1, 0])))


def test_deepest_program():
    # a depth-12 program: a full binary tree of height 12
    rng = synth.rng_for(12)

    def full_c(d):
        if d == 0:
            return "x0" if rng.random() < 0.5 else "%.6f" % rng.uniform(-1, 1)
        op = "+-*"[int(rng.integers(3))]
        return "(%s %s %s)" % (op, full_c(d - 1), full_c(d - 1))
    e = full_c(12)
    tok, cst = progs.parse(e)
    _, st = gp.gp_lower_tree(tok, cst, 1)
    assert st["max_depth"] == 12
    pop = synth.trees_from_lists([(tok, cst)])
    X = synth.uniform_cases(rng, 1, 700, -1, 1)
    say("deepest program")
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert same_bits(got, ref).all()


def test_more_features_than_used():
    rng = synth.rng_for(13)
    pop = synth.ptc2_population(rng, 50, synth.BASIC, 3, 1, 60, 0.2)
    X = synth.uniform_cases(rng, 40, 900, -2, 2)   # 40 features, programs read 3
    say("40-feature matrix")
    got = gpu_tree(pop, X, None, "cases")
    ref = oracle.tree_outputs(pop.tok, pop.cst, pop.off, X)
    assert same_bits(got, ref).all()


def test_errors_are_reported():
    import torch
    X = torch.zeros((2, 10), device="cuda")
    out = torch.zeros(1, device="cuda")
    pop = progs.pop("(+ x0 x1)")
    with pytest.raises(gp.GPError) as e:
        gp.gp_eval_tree(pop.tok, pop.cst, pop.off, X, None, "mse", out)    # y missing
    assert e.value.status == gp.GP_E_INVAL
    with pytest.raises(gp.GPError) as e:
        gp.gp_eval_tree(pop.tok, pop.cst, pop.off, X, out, 7, out)         # bad kind
    assert e.value.status == gp.GP_E_INVAL
    with pytest.raises(gp.GPError):
        gp.gp_eval_tree(pop.tok, pop.cst, pop.off, X, out, "mse", out, n_feat=1)  # x1 >= n_feat


# --------------------------------------------------------------------------
# Register linear programs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_feat,n_cases,n_reg", [(16, 20001, 8), (4, 1000, 8), (1, 130, 3), (30, 515, 8)])
def test_linear_hits_exact(n_feat, n_cases, n_reg):
    rng = synth.rng_for(200 + n_feat)
    pop = synth.linear_population(rng, 150, 20, 200, synth.BASIC, n_reg, n_feat)
    X = synth.normal_cases(rng, n_feat, n_cases)
    _, y = synth.sign_labels(rng, X)
    say("linear F=%d N=%d R=%d: cases" % (n_feat, n_cases, n_reg))
    got = gpu_linear(pop, X, None, "cases")
    ref = oracle.linear_outputs(pop.code, pop.off, pop.cst, pop.cst_off, n_reg, X)
    assert same_bits(got, ref).all()
    say("linear hits")
    got = gpu_linear(pop, X, y, "hits")
    ref = oracle.eval_linear(pop.code, pop.off, pop.cst, pop.cst_off, n_reg, X, y, "hits")
    assert np.array_equal(got, ref)


def test_linear_constants_and_all_ops():
    rng = synth.rng_for(17)
    pop = synth.linear_population(rng, 120, 5, 120, synth.FULL, 8, 6, n_const=5)
    X = synth.uniform_cases(rng, 6, 3000, -3, 3)
    y = synth.gaussian_noise(rng, 3000, 1.0)
    say("linear all ops: cases")
    got = gpu_linear(pop, X, None, "cases")
    ref = oracle.linear_outputs(pop.code, pop.off, pop.cst, pop.cst_off, 8, X)
    tr = np.array([np.any(((pop.code[pop.off[p]:pop.off[p + 1]] & 0xFF) >= 4)) for p in range(pop.n_prog)])
    assert same_bits(got[~tr], ref[~tr]).all()
    say("linear all ops: mse")
    got = gpu_linear(pop, X, y, "mse")
    ref = oracle.eval_linear(pop.code, pop.off, pop.cst, pop.cst_off, 8, X, y, "mse")
    assert fitness_close(got[~tr], ref[~tr]).all()


def test_tree_and_linear_forms_agree_on_gpu():
    rng = synth.rng_for(19)
    pop = synth.ptc2_population(rng, 200, synth.FULL, 5, 2, 100, 0.2)
    codes, consts, keep = [], [], []
    for p in range(pop.n_prog):
        t, c = pop.program(p)
        r = progs.tree_to_register_lgp(t, c, 8)
        if r is not None:
            codes.append(r[0]); consts.append(r[1]); keep.append(p)
    lp = synth.linear_from_lists(codes, consts, 8)
    X = synth.uniform_cases(rng, 5, 1234, -4, 4)
    say("tree vs linear on gpu")
    a = gpu_tree(pop.subset(keep), X, None, "cases")
    b = gpu_linear(lp, X, None, "cases")
    assert same_bits(a, b).all()


# --------------------------------------------------------------------------
# Resident program sets
# --------------------------------------------------------------------------
def test_progset_reuse_and_several_datasets():
    import torch
    rng = synth.rng_for(23)
    pop = synth.ptc2_population(rng, 90, synth.BASIC, 4, 1, 100, 0.2)
    ps = gp.ProgSet.tree(pop.tok, pop.cst, pop.off, 4)
    info = ps.info()
    assert info["n_prog"] == 90 and info["n_gpop"] == len(pop.tok)
    for n in (100, 5000):
        X = synth.uniform_cases(rng, 6, n, -2, 2)
        y = synth.gaussian_noise(rng, n, 1.0)
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        say("progset N=%d" % n)
        o1 = gp.out_tensor("mse", 90, n)
        o2 = gp.out_tensor("mse", 90, n)
        ps.eval(Xd, yd, "mse", o1)
        ps.eval(Xd, yd, "mse", o2)
        torch.cuda.synchronize()
        ref = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, "mse")
        assert torch.equal(o1, o2)
        assert fitness_close(o1.cpu().numpy(), ref).all()
    ps.close()


def test_progset_uploaded_on_one_stream_evaluated_on_another():
    """A program set is uploaded on the stream it is created on; evaluations
    on other streams are ordered after that upload."""
    import torch
    rng = synth.rng_for(29)
    pop = synth.ptc2_population(rng, 300, synth.BASIC, 6, 1, 200, 0.2)
    n = 20000
    X = synth.uniform_cases(rng, 6, n, -2, 2)
    y = synth.gaussian_noise(rng, n, 1.0)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    ref = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, "mse", threads=8)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    # keep stream A busy so that a missing dependency would show
    big = torch.randn(4096, 4096, device="cuda")
    with torch.cuda.stream(sa):
        for _ in range(4):
            big = big @ big * 1e-3
        ps = gp.ProgSet.tree(pop.tok, pop.cst, pop.off, 6, stream=sa)
    outs = []
    for s in (sb, sa, sb):
        o = gp.out_tensor("mse", pop.n_prog, n)
        with torch.cuda.stream(s):
            ps.eval(Xd, yd, "mse", o, stream=s)
        outs.append(o)
    torch.cuda.synchronize()
    say("progset across streams")
    for o in outs:
        assert fitness_close(o.cpu().numpy(), ref).all()
    ps.close()


def test_one_shot_calls_do_not_leak_device_memory():
    """Repeated one-shot evaluations reuse the library's buffers: free device
    memory is the same after 50 more calls."""
    import torch
    rng = synth.rng_for(31)
    pop = synth.ptc2_population(rng, 200, synth.BASIC, 4, 1, 100, 0.2)
    n = 3000
    X = synth.uniform_cases(rng, 4, n, -2, 2)
    y = synth.gaussian_noise(rng, n, 1.0)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    out = gp.out_tensor("mse", pop.n_prog, n)
    for _ in range(5):
        gp.gp_eval_tree(pop.tok, pop.cst, pop.off, Xd, yd, "mse", out)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(50):
        gp.gp_eval_tree(pop.tok, pop.cst, pop.off, Xd, yd, "mse", out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("free device memory before/after 50 calls:", free0, free1)
    assert free1 == free0
    ref = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, "mse")
    assert fitness_close(out.cpu().numpy(), ref).all()


# --------------------------------------------------------------------------
# Full-size workloads, sampled programs
# --------------------------------------------------------------------------
@pytest.mark.slow
def test_full_scale_tree_workload_sampled():
    import torch
    w = synth.scale_tree_workload()
    X = w.X
    say("full scale-tree: target")
    t = None
    for i in range(w.target.n_prog):
        tt = w.target.subset([i])
        v = oracle.tree_outputs(tt.tok, tt.cst, tt.off, X)[0]
        if np.all(np.isfinite(v)) and np.all(np.abs(v) < 1e6):
            t = v
            break
    assert t is not None
    y = (t + w.noise).astype(np.float32)
    say("full scale-tree: gpu 4096 x 65536")
    got = gpu_tree(w.pop, X, y, "mse")
    sample = np.linspace(0, w.pop.n_prog - 1, 24).astype(int)
    sub = w.pop.subset(sample)
    say("full scale-tree: oracle sample")
    ref, ok = well_conditioned_tree(sub, X, y, "mse")
    good = fitness_close(got[sample], ref)
    say("sampled", len(sample), "ill-conditioned", int((~ok).sum()))
    assert good[ok].all(), (sample[ok][~good[ok]], got[sample][ok][~good[ok]], ref[ok][~good[ok]])


@pytest.mark.slow
def test_full_linear_workload_sampled():
    w = synth.linear_workload()
    say("full linear: gpu 4096 x 1M")
    got = gpu_linear(w.pop, w.X, w.y, "hits")
    sample = np.array([0, 1365, 2730, 4095])
    sub = w.pop.subset(sample)
    say("full linear: oracle sample")
    ref = oracle.eval_linear(sub.code, sub.off, sub.cst, sub.cst_off, 8, w.X, w.y, "hits", threads=8)
    assert np.array_equal(got[sample], ref)
    assert np.all((got >= 0) & (got <= w.X.shape[1]))


# --------------------------------------------------------------------------
# Launch shapes: the program grouping and the number of tiles each wave
# walks change the schedule only, never a result
# --------------------------------------------------------------------------
@pytest.mark.parametrize("form", ["tree", "linear"])
def test_launch_shapes_give_identical_results(form, monkeypatch):
    import torch
    rng = synth.rng_for(31)
    F = 8
    if form == "tree":
        pop = synth.ptc2_population(rng, 150, synth.FULL, F, 1, 120, 1 / 9)
    else:
        pop = synth.linear_population(rng, 150, 1, 120, synth.BASIC, 8, F, n_const=2)
    # 14 tiles of 512 cases and a ragged last one: chunks of 4 * tiles_per_wave
    # tiles do not divide it for most shapes
    N = 512 * 13 + 301
    X = synth.uniform_cases(rng, F, N, -3, 3)
    y = synth.gaussian_noise(rng, N, 1.0)
    kind = "mse"
    ref = None
    # (core instructions per group, tiles per wave, blocks the launch aims for)
    for gi, tpw, tb, sg in ((0, 0, 0, 0), (1, 1, 1, 0), (7, 3, 1, 0), (40, 2, 1, 0), (100000, 16, 1, 0),
                            (100000, 1, 1, 0), (192, 5, 1, 0), (192, 0, 4096, 0), (7, 3, 1, 1), (192, 0, 4096, 1),
                            (1, 1, 1, 1)):
        # sg: the four waves of a block run one group on four chunks of tiles
        monkeypatch.setenv("GP2D_SAME_GROUP", str(sg))
        if gi:
            monkeypatch.setenv("GP2D_GROUP_INSTR", str(gi))
            monkeypatch.setenv("GP2D_TARGET_BLOCKS", str(tb))
            if tpw:
                monkeypatch.setenv("GP2D_TILES_PER_WAVE", str(tpw))
            else:
                monkeypatch.delenv("GP2D_TILES_PER_WAVE", raising=False)
        say("launch shape %s group_instr=%d tiles_per_wave=%d target_blocks=%d same_group=%d" % (form, gi, tpw, tb, sg))
        got = gpu_tree(pop, X, y, kind) if form == "tree" else gpu_linear(pop, X, y, kind)
        cases = gpu_tree(pop, X, None, "cases") if form == "tree" else gpu_linear(pop, X, None, "cases")
        if ref is None:
            ref, ref_cases = got, cases
            want = (oracle.tree_outputs(pop.tok, pop.cst, pop.off, X) if form == "tree" else
                    oracle.linear_outputs(pop.code, pop.off, pop.cst, pop.cst_off, pop.n_reg, X))
            assert same_bits(cases, want).mean() >= 0.9999
        assert np.array_equal(got.view(np.int32), ref.view(np.int32))
        assert same_bits(cases, ref_cases).all()
    torch.cuda.synchronize()


def test_forced_variant_is_the_one_reported_and_run(monkeypatch):
    """GP2D_VARIANT (tuning) makes a program set run another kernel variant
    that can hold its programs; the set reports that variant, and fitness
    still matches the oracle.  A value naming no variant leaves the default."""
    import torch
    rng = synth.rng_for(37)
    F, N = 8, 512 * 5 + 77
    pop = synth.ptc2_population(rng, 120, synth.ARITH3, F, 1, 100, 0.2)
    X = synth.uniform_cases(rng, F, N, -2, 2)
    y = synth.gaussian_noise(rng, N, 1.0)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    ref = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, "sum_abs")
    monkeypatch.delenv("GP2D_VARIANT", raising=False)
    ps = gp.ProgSet.tree(pop.tok, pop.cst, pop.off, F)
    info = ps.info()
    base = info["variant"]
    vs = gp.variants()
    alt = [i for i, v in enumerate(vs)
           if i != base and not v["boolean"] and v["n_feat"] >= F and v["depth"] >= info["max_depth"]]
    assert alt
    for vi in sorted({alt[0], alt[-1]}):
        monkeypatch.setenv("GP2D_VARIANT", str(vi + 1))
        assert ps.info()["variant"] == vi
        o = gp.out_tensor("sum_abs", pop.n_prog, N)
        say("forced variant %d (%s)" % (vi, vs[vi]["kernel"]))
        ps.eval(Xd, yd, "sum_abs", o)
        torch.cuda.synchronize()
        assert fitness_close(o.cpu().numpy(), ref).all()
    monkeypatch.setenv("GP2D_VARIANT", str(len(vs) + 1))
    assert ps.info()["variant"] == base
    ps.close()
