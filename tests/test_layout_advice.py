"""Host tests of the layout advisor tc_suggest_layout (Sec. 3.3 and the
closing remarks of Sec. 5: store the inputs so that a free index sits at
stride 1 and GEMM applies without a copy).

The suggested layouts are checked against the brute-force slicing oracle,
which enumerates the slicings of Sec. 2.4 and tests R1-R3 of Sec. 3.1 on its
own: whenever both inputs have a free index, some slicing of the suggested
layout must meet R1, R2 and R3 (Class 3.2).  No GPU needed."""
import ctypes

import numpy as np
import pytest

import paper_1307_2100_amd as tc
import synth
from oracle import slicing


def packed(shape, order=None):
    """Column-major strides with the modes stored in `order` (default: listed)."""
    order = list(range(len(shape))) if order is None else order
    st, acc = [0] * len(shape), 1
    for pos in order:
        st[pos] = acc
        acc *= shape[pos]
    return st


def advise(la, lb, lc, ext, fixed=0, strides=None):
    strides = strides or {}
    ds = [tc.Desc([ext[l] for l in lab], strides.get(n, packed([ext[l] for l in lab])), lab)
          for n, lab in (("A", la), ("B", lb), ("C", lc))]
    return tc.tc_suggest_layout(*ds, fixed=fixed)


def storage_order(strides):
    return sorted(range(len(strides)), key=lambda i: (strides[i], i))


def deltas(la, lb, lc):
    return slicing.delta(list(la), list(lb), list(lc))


def test_examples_from_the_classes():
    ext = {l: 4 for l in "abghij"}
    # Class 3.1 (both stride-1 modes are different contracted indices): the
    # advice moves a free index to stride 1 in both inputs
    (oa, ob, oc), info = advise("gab", "bgh", "ah", ext)
    assert ["gab"[i] for i in oa] == list("agb") and ["bgh"[i] for i in ob] == list("gbh")
    assert ["ah"[i] for i in oc] == list("ah")
    assert info.paper_class == 32 and info.recipe == tc.TC_RECIPE_GEMM and info.copy_operand == -1
    assert (info.nM, info.nN, info.nK) == (1, 1, 1)
    # the convenience form on label strings
    out, info = tc.suggest_layout("gab", [4, 4, 4], "bgh", [4, 4, 4], "ah", [4, 4])
    assert out == {"A": "agb", "B": "gbh", "C": "ah"} and info.paper_class == 32
    # A kept as given: B leads with its free index instead
    out, info = tc.suggest_layout("gab", [4, 4, 4], "bgh", [4, 4, 4], "ah", [4, 4], fixed="A")
    assert out["A"] == "gab" and out["B"][0] == "h" and info.paper_class == 32
    # both inputs kept: the class cannot change
    out, info = tc.suggest_layout("gab", [4, 4, 4], "bgh", [4, 4, 4], "ah", [4, 4], fixed="AB")
    assert out["A"] == "gab" and out["B"] == "bgh" and info.paper_class == 31
    # Class 2 and 1 stay what they are: Delta does not depend on the layout
    _, info = advise("abg", "bg", "a", ext)
    assert info.paper_class == 2
    _, info = advise("abg", "gab", "", ext)
    assert info.paper_class == 1


def test_table_new3d_every_layout_becomes_class_32():
    """The 18 layouts of the 3-D square experiments (4 of them Class 3.1):
    the suggestion is Class 3.2 for every one, by the oracle's R1-R3 test."""
    ext = {l: 5 for l in "abgh"}
    for con in (("b", "g"), ("a", "g"), ("a", "b")):
        free_a = [l for l in "abg" if l not in con][0]
        for order in (con, con[::-1]):
            for pos in (2, 1, 0):
                lb = list(order)
                lb.insert(pos, "h")
                lb = "".join(lb)
                lc = free_a + "h"
                (oa, ob, oc), info = advise("abg", lb, lc, ext)
                sa = ["abg"[i] for i in oa]
                sb = [lb[i] for i in ob]
                assert slicing.classify(sa, sb, 0, 0, list(lc)) == 32
                assert slicing.gemm_slicings(sa, sb, 0, 0, list(lc))
                assert info.paper_class == 32 and info.recipe == tc.TC_RECIPE_GEMM


@pytest.mark.parametrize("fixed", [0, 1, 2, 4, 3, 5, 6, 7])
def test_random_contractions_against_the_slicing_oracle(fixed):
    g = np.random.default_rng(1307 + fixed)
    seen = set()
    for _ in range(400):
        la, lb, lc, ext = synth.random_contraction(g, rank_range=(1, 5), ext_range=(2, 4),
                                                   max_elems=10 ** 9, p_outer=0.05, allow_batch=True)
        strides, stor = {}, {}
        for name, labs in (("A", la), ("B", lb), ("C", lc)):
            order = list(g.permutation(len(labs)))
            strides[name] = packed([ext[l] for l in labs], order)
            stor[name] = storage_order(strides[name])
        (oa, ob, oc), info = advise(la, lb, lc, ext, fixed=fixed, strides=strides)
        for bit, (name, labs, o) in enumerate((("A", la, oa), ("B", lb, ob), ("C", lc, oc))):
            assert sorted(o) == list(range(len(labs)))          # a permutation of the listed modes
            if fixed & (1 << bit):
                assert o == stor[name]                          # a fixed tensor keeps its storage
        sa, sb, sc = [la[i] for i in oa], [lb[i] for i in ob], [lc[i] for i in oc]
        got = slicing.classify(sa, sb, 0 if sa else None, 0 if sb else None, sc)
        assert info.paper_class == got, (la, lb, lc, fixed)
        dA, dB, p = deltas(la, lb, lc)
        given = slicing.classify([la[i] for i in stor["A"]], [lb[i] for i in stor["B"]],
                                 0 if la else None, 0 if lb else None, lc)
        if p == 0 or dA == 0 or dB == 0:
            assert got == given                                 # Classes 0, 1, 2 do not depend on storage
        elif (fixed & 3) == 3:
            assert got == given                                 # both inputs kept
        elif ((fixed & 1) and sa[0] in set(lc) and sa[0] in set(lb)) or \
                ((fixed & 2) and sb[0] in set(lc) and sb[0] in set(la)):
            assert got == 31                                    # a kept input has a batch index at stride 1
        else:
            assert got == 32, (la, lb, lc, fixed, sa, sb)
            assert info.recipe == tc.TC_RECIPE_GEMM and info.copy_operand == -1
            if fixed == 0:
                # one order per group in every tensor: each group fuses to one mode
                assert max(info.nM, info.nN, info.nK, info.nL) <= 1
        seen.add(got)
    assert 32 in seen


def test_errors():
    ext = {l: 3 for l in "abc"}
    d = lambda lab: tc.Desc([ext[l] for l in lab], packed([ext[l] for l in lab]), lab)
    with pytest.raises(tc.TCError) as e:
        tc.tc_suggest_layout(d("ab"), d("bc"), d("ac"), fixed=8)
    assert e.value.status == tc.TC_ERR_INVALID_ARG
    with pytest.raises(tc.TCError) as e:
        tc.tc_suggest_layout(d("ab"), d("cb"), d("a"), fixed=0)   # c appears in B only
    assert e.value.status == tc.TC_ERR_LABEL
    bad = tc.Desc([3, 4], [1, 3], "bc")
    with pytest.raises(tc.TCError) as e:
        tc.tc_suggest_layout(d("ab"), bad, d("ac"), fixed=0)
    assert e.value.status == tc.TC_ERR_EXTENT_MISMATCH
    # a null order array is rejected before anything is written
    oa = (ctypes.c_int32 * 2)(-7, -7)
    st = tc._lib.tc_suggest_layout(*d("ab").args(), *d("bc").args(), *d("ac").args(), 0, oa, None, None, None)
    assert st == tc.TC_ERR_INVALID_ARG and list(oa) == [-7, -7]
    # stride arrays may be NULL: packed in the listed order
    oa, ob, oc = [(ctypes.c_int32 * 2)() for _ in range(3)]
    A, B, C = d("ba"), d("bc"), d("ac")
    st = tc._lib.tc_suggest_layout(A.rank, A.ext, None, A.lab, B.rank, B.ext, None, B.lab, C.rank, C.ext, None,
                                   C.lab, 1, oa, ob, oc, None)
    assert st == tc.TC_OK and list(oa) == [0, 1] and list(ob) == [1, 0]
