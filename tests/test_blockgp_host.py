"""Host-side checks of the one-dimensional-stack comparator's entry point
(gp_eval_tree_1d): malformed requests are rejected before anything touches
the device, so these run without a GPU."""
import ctypes as C

import numpy as np
import pytest

import paper_1601_00221_amd as gp
import synth
from tests import progs

FAKE = C.c_void_p(256)   # never dereferenced: every call below fails validation first


def call(pop, form, n_feat=3, kind=gp.GP_OUT_CASES):
    tok = np.ascontiguousarray(pop.tok, np.int32)
    cst = np.ascontiguousarray(pop.cst, np.float32)
    off = np.ascontiguousarray(pop.off, np.int64)
    return gp.lib().gp_eval_tree_1d(tok.ctypes.data_as(C.c_void_p), cst.ctypes.data_as(C.c_void_p),
                                    off.ctypes.data_as(C.c_void_p), len(off) - 1, FAKE, n_feat, 8, FAKE,
                                    kind, form, FAKE, None)


def test_exported():
    assert hasattr(gp.lib(), "gp_eval_tree_1d")


def test_unknown_form_and_kind():
    pop = progs.pop("(+ x0 x1)")
    assert call(pop, 2) == gp.GP_E_INVAL
    assert call(pop, -1) == gp.GP_E_INVAL
    assert call(pop, 0, kind=7) == gp.GP_E_INVAL


def test_feature_out_of_range():
    pop = progs.pop("(+ x0 x5)")
    assert call(pop, 0, n_feat=3) == gp.GP_E_INVAL
    assert "feature" in gp.last_error()


def test_postfix_stack_limit():
    # (+ x0 (+ x0 ... x0)) with k additions needs k + 1 postfix stack values
    deep = "x0"
    for _ in range(64):
        deep = "(+ x0 %s)" % deep
    assert call(progs.pop(deep), gp.GP_1D_FORMS["rpn"]) == gp.GP_E_DEPTH
    assert "stack" in gp.last_error()


@pytest.mark.parametrize("form", ["rpn", "lgp"])
def test_length_limit(form):
    # 4097 nested sines: 4098 nodes, 4097 stack-operand instructions
    tok = np.array([synth.SIN] * 4097 + [synth.var_tok(0)], np.int32)
    pop = synth.trees_from_lists([(tok, np.zeros(len(tok), np.float32))])
    assert call(pop, gp.GP_1D_FORMS[form]) == gp.GP_E_DEPTH
