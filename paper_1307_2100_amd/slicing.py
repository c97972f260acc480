"""Forced slicings: a contraction run as the paper's slice loops.

Sec. 2.4 turns a contraction into loops over its *sliced* indices around one
BLAS call per slice; which call depends on what stays unsliced (two matrices
-> GEMM, a matrix and a vector -> GEMV, two vectors -> DOT or GER).  The
library normally fuses every sliced index into one launch; this module runs
a chosen slicing verbatim instead, to compare the two:

    run_sliced(A, "abg", B, "hbg", C, "ah", sliced="g")   # n GEMMs, C accumulated

Every label in `sliced` becomes a loop index.  A sliced contracted index is
sliced in both inputs (the remark under R2 in Sec. 3.1) and its slices are
accumulated into C in index order: the first with the caller's beta, the
rest with beta = 1.  A sliced free or batch index selects the matching slice
of C.  One libtc plan covers every slice (the slices share extents and
strides; only their base addresses differ), so each slice is one tc_execute
call: the recipe of the slice's own class, or the one forced by `recipe`.
"""
import itertools

from . import Plan, labels_of


def _select(t, lab, fixed):
    """View of tensor t (labels lab) with the labels in `fixed` held at their
    values; returns (view, remaining labels)."""
    keep = []
    for pos in range(len(lab) - 1, -1, -1):
        if lab[pos] in fixed:
            t = t.select(pos, fixed[lab[pos]])
    for l in lab:
        if l not in fixed:
            keep.append(l)
    return t, keep


def slice_count(A, labA, B, labB, sliced):
    """Number of slices (library calls) a slicing takes."""
    ext = dict(zip(labels_of(labA), A.shape))
    ext.update(zip(labels_of(labB), B.shape))
    n = 1
    for l in labels_of(sliced):
        n *= ext[l]
    return n


def run_sliced(A, labA, B, labB, C, labC, sliced, alpha=1.0, beta=0.0, recipe="auto", stream=None):
    """C <- alpha * sum A*B + beta * C as loops over the labels in `sliced`
    with one library call per slice.  Returns the number of calls."""
    la, lb, lc, ls = (labels_of(x) for x in (labA, labB, labC, sliced))
    ext = dict(zip(la, A.shape))
    ext.update(zip(lb, B.shape))
    for l in ls:
        if l not in ext:
            raise ValueError("sliced label %r is in neither input" % (l,))
        if ext[l] < 1:
            raise ValueError("sliced label %r has extent 0" % (l,))
    if len(set(ls)) != len(ls):
        raise ValueError("a label is sliced twice")
    contracted = [l for l in ls if l in la and l in lb and l not in lc]
    outer = [l for l in ls if l not in contracted]
    calls = 0
    plan = None
    try:
        for oidx in itertools.product(*[range(ext[l]) for l in outer]):
            fixed = dict(zip(outer, oidx))
            first = True
            for cidx in itertools.product(*[range(ext[l]) for l in contracted]):
                f = dict(fixed)
                f.update(zip(contracted, cidx))
                As, sa = _select(A, la, f)
                Bs, sb = _select(B, lb, f)
                Cs, sc = _select(C, lc, f)
                if plan is None:
                    plan = Plan.for_tensors(As, sa, Bs, sb, Cs, sc, recipe=recipe)
                plan.execute(As, Bs, Cs, alpha, beta if first else 1.0, stream=stream)
                first = False
                calls += 1
    finally:
        if plan is not None:
            # the plan's tables and workspace must outlive the enqueued calls
            import torch
            (stream or torch.cuda.current_stream()).synchronize()
            plan.close()
    return calls
