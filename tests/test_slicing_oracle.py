"""Pins of the brute-force slicing oracle against the paper's own examples
(Sec. 2.4, Sec. 3.2, Table tab:new3D, Eq. (xy)) and the Class-3.1 definition."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import slicing

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIX = json.load(open(os.path.join(GOLDEN, "paper_slicings.json")))


@pytest.mark.parametrize("case", FIX["cases"], ids=[c["where"][:40] for c in FIX["cases"]])
def test_paper_slicing_kernels(case):
    found = [s for s in slicing.enumerate_slicings(case["T"], case["S"], 0, 0, case["R"] or None)
             if s["sT"] == tuple(case["sT"]) and s["sS"] == tuple(case["sS"])]
    assert len(found) == 1, "slicing vectors are not consistent on contracted labels"
    assert found[0]["kernel"] == case["kernel"]


@pytest.mark.parametrize("case", FIX["classes"], ids=[c["where"][:40] for c in FIX["classes"]])
def test_paper_classes(case):
    assert slicing.classify(case["T"], case["S"], 0, 0, case["R"] or None) == case["class"]


def test_paper_requirements_on_examples():
    # Sec. 2.4 (a) satisfies R1-R3; (b) breaks R1 only (F1); (c) breaks R2 (F2)
    # S^{sr} stays unsliced in all three examples
    sl = {s["sT"]: s for s in slicing.enumerate_slicings("abs", "sr", 0, 0, "abr") if s["sS"] == (0, 0)}
    assert sl[(0, 1, 0)]["R1"] and sl[(0, 1, 0)]["R2"] and sl[(0, 1, 0)]["R3"]
    assert not sl[(1, 0, 0)]["R1"] and sl[(1, 0, 0)]["R2"] and sl[(1, 0, 0)]["R3"]
    assert not sl[(1, 1, 0)]["R2"]
    # F3 example: s(T) = (0,0,1) slices the only contracted index: no BLAS-3 or -2 kernel
    f3 = [s for s in slicing.enumerate_slicings("abs", "sr", 0, 0, "abr") if s["sT"] == (0, 0, 1)]
    assert f3 and all(s["kernel"] is None for s in f3)
    # Eq. (xy)(a): s(X)=s(Y)=(0,0,1,1) satisfies all three requirements
    ok = [s for s in slicing.gemm_slicings("iajb", "igjd", 0, 0, "abgd")]
    assert ((0, 0, 1, 1), (0, 0, 1, 1)) in [(s["sT"], s["sS"]) for s in ok]
    # Fig. 3D-2: both slicings of A^{abg}B_{hbg} lead to GEMM
    g = [(s["sT"], s["sS"]) for s in slicing.gemm_slicings("abg", "hbg", 0, 0, "ah")]
    assert set(g) == {((0, 1, 0), (0, 1, 0)), ((0, 0, 1), (0, 0, 1))}


def _table_new3d():
    """The 18 double contractions of Table tab:new3D: A^{abg} with two of its
    labels contracted against B, B's free label h in 3rd, 2nd or 1st place."""
    out = []
    for con in (("b", "g"), ("a", "g"), ("a", "b")):
        free_a = [l for l in "abg" if l not in con][0]
        for order in (con, con[::-1]):
            for pos in (2, 1, 0):
                lb = list(order)
                lb.insert(pos, "h")
                out.append(("abg", "".join(lb), free_a + "h"))
    return out


def test_table_new3d_follows_class_definition():
    """Class 3.1 holds exactly when the stride-1 (first) indices of A and B are
    distinct and both contracted (Sec. 3.2); the highlighted cases are 3.1 and 3.2."""
    rows = _table_new3d()
    assert len(rows) == 18 and len(set(r[1] for r in rows)) == 18
    counts = {31: 0, 32: 0}
    for la, lb, lc in rows:
        cls = slicing.classify(la, lb, 0, 0, lc)
        rule = 31 if (la[0] != lb[0] and la[0] in lb and lb[0] in la) else 32
        assert cls == rule, (la, lb)
        counts[cls] += 1
    # The paper's text counts 12 + 4 for the 16 non-highlighted cases; the
    # definition gives 3 + 13 of those (4 + 14 of all 18).  The definition wins.
    assert counts == {31: 4, 32: 14}


def _rule_class(labA, labB, labC, unitA, unitB):
    batch = set(labA) & set(labB) & set(labC)
    con = [l for l in labA if l in labB and l not in batch]
    p = len(con)
    dA = len([l for l in labA if l not in batch]) - p
    dB = len([l for l in labB if l not in batch]) - p
    if p == 0:
        return 0
    if dA == 0 and dB == 0:
        return 1
    if dA == 0 or dB == 0:
        return 2
    if unitA is None or unitB is None:
        return 31
    ua, ub = labA[unitA], labB[unitB]
    if ua in batch or ub in batch:      # batch labels are always sliced: no unit-stride slice
        return 31
    return 31 if (ua != ub and ua in con and ub in con) else 32


def test_constructive_class_equals_stride_rule_on_random_shapes():
    """Over 3000 random contractions (ranks 1-5, random storage order and
    stride-1 position, sometimes none), 'some slicing meets R1-R3' coincides with
    the paper's stride-1 rule for Class 3."""
    g = np.random.default_rng(2024)
    seen = set()
    for _ in range(3000):
        la, lb, lc, ext = synth.random_contraction(g, rank_range=(1, 5), ext_range=(2, 3),
                                                   max_elems=10 ** 9, p_outer=0.05, allow_batch=True)
        ua = None if g.random() < 0.05 else int(g.integers(len(la)))
        ub = None if g.random() < 0.05 else int(g.integers(len(lb)))
        want = _rule_class(la, lb, lc, ua, ub)
        got = slicing.classify(la, lb, ua, ub, lc)
        assert got == want, (la, lb, lc, ua, ub)
        seen.add(got)
    assert seen == {0, 1, 2, 31, 32}
