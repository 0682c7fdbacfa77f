"""Runs the library's host paths and the oracle, built with the address and
undefined-behaviour sanitizers, on random and malformed input (no device).

    python sanitize_exercise.py LIBGP_SANITIZED LIBORACLE_SANITIZED

Started by tests/test_sanitized_host.py with the sanitizer runtime preloaded;
any sanitizer report ends the process with a nonzero status."""
import ctypes as C
import os
import sys
import threading

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                      # noqa: E402
import paper_1601_00221_amd as gp  # noqa: E402
import synth                       # noqa: E402

gp.LIB_PATH = sys.argv[1]
oracle.LIB = sys.argv[2]


def lowering_and_translation(rng):
    fsets = [synth.FULL, synth.SHUTTLE_SET, synth.KDD_SET, synth.ARITH3]
    for k, fs in enumerate(fsets):
        pop = synth.ptc2_population(rng, 120, fs, 9, 1, 300, 0.2)
        for p in range(0, pop.n_prog, 3):
            t, c = pop.program(p)
            gp.gp_lower_tree(t, c, 9)
        for vi, v in enumerate(gp.variants()):
            if v["boolean"] or v["n_feat"] < 9:
                continue
            try:
                gp.core_lower(pop, 9, vi, 0x7F0000000000)
            except gp.GPError:
                pass      # too deep for the variant, or transcendentals on a kernel without them
    lin = synth.linear_population(rng, 80, 1, 200, synth.BASIC + (synth.GT, synth.AND), 8, 12, n_const=3)
    for vi, v in enumerate(gp.variants()):
        if not v["trees_only"] and not v["boolean"] and v["n_feat"] >= 12:
            gp.core_lower(lin, 12, vi, 0x7F0000000000)
    # malformed programs: every one must be rejected with an error, never read out of bounds
    bad = [np.array([synth.ADD], np.int32), np.array([synth.VAR | (50 << 8)], np.int32),
           np.array([synth.IF, synth.CONST, synth.CONST], np.int32), np.array([200, 1, 2], np.int32),
           np.array([synth.SIN, synth.CONST, synth.CONST], np.int32)]
    for t in bad:
        try:
            gp.gp_lower_tree(t, np.zeros(len(t), np.float32), 9)
        except gp.GPError:
            continue
        raise AssertionError("accepted a malformed tree")
    for _ in range(300):
        n = int(rng.integers(1, 40))
        t = rng.choice([0, 1, 2, 3, 4, 7, 8, 12, 15, 64, 65, 64 | (3 << 8), 99], n).astype(np.int32)
        try:
            gp.gp_lower_tree(t, rng.standard_normal(n).astype(np.float32), 4)
        except gp.GPError:
            pass


def breeding(rng):
    for fs, kind in ((synth.FULL, "mse"), (synth.SHUTTLE_SET, "class_err"), (synth.BOOL_SET, "hits")):
        cfg = gp.evolve_config(fs, kind=kind, pop_size=150, max_size=200, max_depth=12, p_const=0.0 if
                               fs == synth.BOOL_SET else 0.2, seed=int(rng.integers(1 << 30)))
        tok, cst, off = gp.init_population(cfg, 6)
        for g in range(3):
            tok, cst, off = gp.breed(cfg, tok, cst, off, 6, rng.random(150), g + 1)


def serving(rng):
    srv = gp.Server(dry_run=True, dry_run_gpops=5e11, memory_budget=8 << 20, max_queue=64)
    # device addresses are never touched in a dry run: stand-ins will do
    ds = [srv.add_dataset(0x10000 + 0x1000 * k, 0x90000 + 0x1000 * k, n_feat=9, n_cases=4096) for k in range(3)]
    pool = synth.ptc2_population(rng, 200, synth.FULL, 9, 1, 200, 0.2)
    lin = synth.linear_population(rng, 200, 1, 100, synth.BASIC, 8, 9)
    errors = []

    def client(k):
        try:
            r = synth.rng_for(100 + k)
            for i in range(12):
                P = int(r.integers(1, 60))
                src = pool if i % 2 == 0 else lin
                pop = synth.pool_slice(src, int(r.integers(200)), P)
                t = srv.submit(gp.make_job(pop, ds[i % 3], "mse", 0x20000))
                if i % 5 == 4:
                    try:
                        srv.cancel(t)
                    except gp.GPError:
                        pass
                srv.wait(t, 10_000_000)
                srv.release(t)
        except Exception as e:   # reported after the join
            errors.append(repr(e))
    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    srv.stats()
    srv.close()
    assert not errors, errors[0]


def oracle_paths(rng):
    for fs in (synth.FULL, synth.SHUTTLE_SET):
        pop = synth.ptc2_population(rng, 40, fs, 5, 1, 120, 0.2)
        X = synth.uniform_cases(rng, 5, 300, -3, 3)
        y = synth.gaussian_noise(rng, 300, 1.0)
        for kind in ("mse", "sum_abs", "hits", "class_err", "cases"):
            oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, kind, threads=3)
    lin = synth.linear_population(rng, 40, 1, 100, synth.BASIC, 8, 5, n_const=2)
    oracle.eval_linear(lin.code, lin.off, lin.cst, lin.cst_off, 8, X, y, "hits", threads=2)
    t, c = synth.ptc2_tree(rng, 50, synth.FULL, 5, 0.2)
    rt, rc = oracle.prefix_to_rpn(t, c)
    oracle.rpn_eval(rt, rc, X, 3)
    ins, m = oracle.rpn_to_lgp(rt, rc)
    oracle.lgp_eval(ins, m, X, 3)


def main():
    rng = synth.rng_for(2024)
    lowering_and_translation(rng)
    breeding(rng)
    serving(rng)
    oracle_paths(rng)
    print("sanitized host paths: ok", flush=True)


if __name__ == "__main__":
    main()
