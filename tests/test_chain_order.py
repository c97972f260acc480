"""Host tests of the chain planner (paper_1307_2100_amd.chain): the pairwise
order it picks has the least flop count over every binary tree, checked by
brute force here, and matches the textbook matrix-chain optimum."""
import itertools

import pytest

from paper_1307_2100_amd import chain, labels_of


def trees(items):
    """Every full binary tree over the items (as nested pairs)."""
    if len(items) == 1:
        yield items[0]
        return
    for r in range(1, len(items)):
        for left in itertools.combinations(items, r):
            right = tuple(x for x in items if x not in left)
            if left[0] != items[0]:
                continue   # each unordered split once
            for a in trees(left):
                for b in trees(right):
                    yield (a, b)


def tree_cost(t, labels, out, ext):
    """(flops, result labels) of a tree: a label survives a step when it is
    in the output or in an operand outside the subtree."""
    def leaves(x):
        return [x] if isinstance(x, int) else leaves(x[0]) + leaves(x[1])

    def rec(x):
        if isinstance(x, int):
            return 0.0, set(labels[x])
        fa, la = rec(x[0])
        fb, lb = rec(x[1])
        inside = set(leaves(x))
        outside = set(out)
        for i, lab in enumerate(labels):
            if i not in inside:
                outside |= set(lab)
        f = 2.0
        for l in la | lb:
            f *= ext[l]
        return fa + fb + f, {l for l in la | lb if l in outside}

    return rec(t)[0]


def test_textbook_matrix_chain():
    # six matrices 30x35, 35x15, 15x5, 5x10, 10x20, 20x25: the classic optimum
    # is 15125 scalar multiplications, ((A1 (A2 A3)) ((A4 A5) A6))
    dims = [30, 35, 15, 5, 10, 20, 25]
    names = "abcdefg"
    labels = [labels_of(names[i] + names[i + 1]) for i in range(6)]
    ext = {ord(names[i]): d for i, d in enumerate(dims)}
    steps, flops = chain.plan_order(labels, labels_of("ag"), ext)
    assert flops == 2 * 15125 and len(steps) == 5
    _, left = chain.plan_order(labels, labels_of("ag"), ext, order="left")
    assert left > flops


@pytest.mark.parametrize("spec", [
    ("abcd,ae,bf->efcd", {"a": 6, "b": 5, "c": 4, "d": 3, "e": 7, "f": 2}),
    ("ij,jk,kl,lm->im", {"i": 9, "j": 2, "k": 30, "l": 3, "m": 11}),
    ("aix,ibx,bcx,c->ax", {"a": 4, "i": 6, "b": 5, "c": 7, "x": 3}),
    ("ab,bc,cd,de,ea->", {"a": 3, "b": 8, "c": 2, "d": 9, "e": 4}),
    ("pq,qrs,st,trp,u->u", {"p": 3, "q": 4, "r": 2, "s": 5, "t": 6, "u": 2}),
])
def test_optimal_order_is_the_least_flop_tree(spec):
    expr, e = spec
    ins, out = expr.split("->")
    labels = [labels_of(x) for x in ins.split(",")]
    ext = {ord(k): v for k, v in e.items()}
    steps, flops = chain.plan_order(labels, labels_of(out), ext)
    best = min(tree_cost(t, labels, labels_of(out), ext) for t in trees(tuple(range(len(labels)))))
    assert flops == best
    assert len(steps) == len(labels) - 1


def test_metric_raising_avoids_the_outer_product():
    ext = {ord(c): 50 for c in "abcdef"}
    labels = [labels_of("ae"), labels_of("bf"), labels_of("abcd")]
    _, opt = chain.plan_order(labels, labels_of("efcd"), ext)
    _, left = chain.plan_order(labels, labels_of("efcd"), ext, order="left")
    assert opt == 2 * 2 * 50 ** 5 and left == 2 * 50 ** 4 + 2 * 50 ** 6


def test_label_rules():
    with pytest.raises(ValueError):
        chain.check_labels([labels_of("ab"), labels_of("bc"), labels_of("bd")], labels_of("acd"))  # b thrice
    with pytest.raises(ValueError):
        chain.check_labels([labels_of("ab"), labels_of("cd")], labels_of("abz"))
    with pytest.raises(ValueError):
        chain.check_labels([labels_of("aa"), labels_of("a")], labels_of(""))
    chain.check_labels([labels_of("abx"), labels_of("bcx"), labels_of("cdx")], labels_of("adx"))
