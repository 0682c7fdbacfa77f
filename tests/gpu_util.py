"""Shared helpers for the GPU parity tests."""
import sys

import numpy as np

import oracle
import paper_1601_00221_amd as gp

TOL_REL = 1e-5          # fitness sums (relative)
ULP_TRANSC = 2          # per-operation bound for sin, cos, exp, log


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_tree(pop, X, y, kind, n_feat=None):
    import torch
    Xd = dev(X)
    yd = dev(y) if y is not None else None
    out = gp.out_tensor(kind, pop.n_prog, X.shape[1])
    gp.gp_eval_tree(pop.tok, pop.cst, pop.off, Xd, yd, kind, out, n_feat=n_feat)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_linear(pop, X, y, kind, n_feat=None):
    import torch
    Xd = dev(X)
    yd = dev(y) if y is not None else None
    out = gp.out_tensor(kind, pop.n_prog, X.shape[1])
    gp.gp_eval_linear(pop.code, pop.off, pop.cst, pop.cst_off, pop.n_reg, Xd, yd, kind, out, n_feat=n_feat)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def ulp_dist(a, b):
    a = np.asarray(a, np.float32); b = np.asarray(b, np.float32)
    ia = a.view(np.int32).astype(np.int64); ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    d = np.abs(ia - ib)
    return np.where(np.isnan(a) & np.isnan(b), 0, d)


def same_bits(a, b):
    a = np.asarray(a, np.float32); b = np.asarray(b, np.float32)
    return (a.view(np.int32) == b.view(np.int32)) | (np.isnan(a) & np.isnan(b))


def fitness_close(got, ref, tol=TOL_REL):
    """Relative closeness with non-finite values matched by class."""
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    fin = np.isfinite(ref) & np.isfinite(got)
    ok = np.zeros(got.shape, bool)
    ok[fin] = np.abs(got[fin] - ref[fin]) <= tol * np.maximum(np.abs(ref[fin]), 1e-30)
    ok |= np.isnan(got) & np.isnan(ref)
    ok |= np.isinf(got) & np.isinf(ref) & (np.sign(got) == np.sign(ref))
    return ok


def has_transcendental_tree(pop):
    out = np.zeros(pop.n_prog, bool)
    for p in range(pop.n_prog):
        t, _ = pop.program(p)
        ops = t & 0xFF
        out[p] = bool(np.any((ops >= 4) & (ops <= 7)))
    return out


def well_conditioned_tree(pop, X, y, kind, margin=TOL_REL):
    """True where moving every sin/cos/exp/log result by +-2 units in the
    last place changes the oracle fitness by at most `margin` relative: a
    program whose fitness depends on the last bits of a transcendental is
    not reproducible by any implementation within the 2-ulp contract."""
    f0 = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, kind, nudge=0, threads=8)
    fp = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, kind, nudge=2, threads=8)
    fm = oracle.eval_tree(pop.tok, pop.cst, pop.off, X, y, kind, nudge=-2, threads=8)
    ok = fitness_close(fp, f0, margin) & fitness_close(fm, f0, margin)
    return f0, ok
