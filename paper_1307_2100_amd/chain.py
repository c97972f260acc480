"""Contractions of several tensors as a sequence of binary contractions.

The appendix of the paper raises and lowers the indices of a tensor with the
metric, one index at a time: T g g ... is a chain of binary contractions,
each of which is the operation of Sec. 2.3.  This module evaluates such
chains with libtc:

    R = contract_chain([(T, "abcd"), (g, "ae"), (g, "bf")], "efcd")

A label summed over must appear in exactly two operands (a repeated index
pair, App. A); a label of the result must appear in at least one operand;
labels shared by more than two operands must also be in the result (they
act as batch indices).  The pairwise order minimises the total flop count
over all binary trees (dynamic programming over subsets of operands, up to
12 operands), or follows the operand order with order="left".  Chain plans
once (order, intermediates, one libtc plan per step) and executes many
times; contract_chain does both for one call.  Each
intermediate is stored in the order tc_suggest_layout gives for an output
whose inputs are fixed (free indices of the first input, then of the second,
then batch indices), column-major; the last step writes the result in the
requested label order.
"""
from . import Plan, _torch, empty_colmajor, labels_of, suggest_layout


def _flops(la, lb, ext):
    """2 x product of the extents of every label of the two inputs."""
    f = 2.0
    for l in set(la) | set(lb):
        f *= ext[l]
    return f


def _result_labels(la, lb, keep):
    """Labels of the binary result: those of either input still needed."""
    out = []
    for l in list(la) + list(lb):
        if l in keep and l not in out:
            out.append(l)
    return out


def plan_order(labels, out, ext, order="optimal"):
    """Pairwise order for operands with these label lists: a list of steps
    (i, j) over a working list (step k contracts entries i < j and appends
    the result, removing both), and the total flop count."""
    n = len(labels)
    if order == "left":
        # ((T0 T1) T2) ...: the running result sits at the end of the list
        steps, cur, flops = [], [list(l) for l in labels], 0.0
        while len(cur) > 1:
            i, j = (0, 1) if not steps else (0, len(cur) - 1)
            rest = [l for k, x in enumerate(cur) if k not in (i, j) for l in x]
            r = _result_labels(cur[i], cur[j], set(rest) | set(out))
            flops += _flops(cur[i], cur[j], ext)
            steps.append((i, j))
            cur = [x for k, x in enumerate(cur) if k not in (i, j)] + [r]
        return steps, flops
    if order != "optimal":
        raise ValueError("order must be 'optimal' or 'left'")
    if n > 12:
        raise ValueError("at most 12 operands for the optimal order")
    full = (1 << n) - 1
    # labels of the subset result: those of the subset also outside it or in the output
    lab_of = {}
    for s in range(1, full + 1):
        inside = set()
        outside = set(out)
        for i in range(n):
            (inside if s >> i & 1 else outside).update(labels[i])
        lab_of[s] = [l for l in inside if l in outside]
    best = {1 << i: (0.0, None) for i in range(n)}
    for s in sorted(range(1, full + 1), key=lambda x: bin(x).count("1")):
        if s in best:
            continue
        b = (float("inf"), None)
        sub = (s - 1) & s
        while sub:
            other = s ^ sub
            if sub < other:   # each split once
                c = best[sub][0] + best[other][0] + _flops(lab_of[sub], lab_of[other], ext)
                if c < b[0]:
                    b = (c, (sub, other))
            sub = (sub - 1) & s
        best[s] = b
    # flatten the tree into steps over a working list
    steps = []
    work = [1 << i for i in range(n)]

    def emit(s):
        if s in work:
            return
        a, c = best[s][1]
        emit(a)
        emit(c)
        i, j = sorted((work.index(a), work.index(c)))
        steps.append((i, j))
        work.pop(j)
        work.pop(i)
        work.append(s)

    emit(full)
    return steps, best[full][0]


def check_labels(labels, out):
    count = {}
    for lab in labels:
        if len(set(lab)) != len(lab):
            raise ValueError("a label repeats within one operand")
        for l in lab:
            count[l] = count.get(l, 0) + 1
    for l, c in count.items():
        if l not in out and c != 2:
            raise ValueError("label %r is summed over but appears in %d operand(s), not 2" % (l, c))
    for l in out:
        if l not in count:
            raise ValueError("output label %r is in no operand" % (l,))
    if len(set(out)) != len(out):
        raise ValueError("an output label repeats")


class Chain:
    """A planned chain: the pairwise order, the intermediates (allocated once)
    and one libtc plan per step, built for operands of these shapes and
    strides.  execute() runs the steps on the current stream; operands of
    later calls must have the same shapes and strides."""

    def __init__(self, operands, out_labels, order="optimal", out=None):
        if len(operands) < 2:
            raise ValueError("a chain needs at least two operands")
        tens = [t for t, _ in operands]
        self.labels = [labels_of(l) for _, l in operands]
        self.out_labels = labels_of(out_labels)
        check_labels(self.labels, self.out_labels)
        ext = {}
        for t, lab in zip(tens, self.labels):
            for l, e in zip(lab, t.shape):
                if ext.setdefault(l, e) != e:
                    raise ValueError("label %r has extents %d and %d" % (l, ext[l], e))
        self.steps, self.flops = plan_order(self.labels, self.out_labels, ext, order)
        # work entries: ("in", k) for operand k, ("tmp", s) for the result of step s
        work = [(("in", k), t, lab) for k, (t, lab) in enumerate(zip(tens, self.labels))]
        self.plans, self.buffers, self.wiring = [], [], []
        try:
            for s_idx, (i, j) in enumerate(self.steps):
                (ka, A, la), (kb, B, lb) = work[i], work[j]
                rest = [l for idx, (_, _, x) in enumerate(work) if idx not in (i, j) for l in x]
                if s_idx == len(self.steps) - 1:
                    lc = self.out_labels
                    C = out if out is not None else empty_colmajor([ext[l] for l in lc], device=A.device)
                else:
                    lc = _result_labels(la, lb, set(rest) | set(self.out_labels))
                    if lc:
                        adv, _ = suggest_layout(la, list(A.shape), lb, list(B.shape), lc, [ext[l] for l in lc],
                                                fixed="AB", strides={"A": list(A.stride()), "B": list(B.stride())})
                        lc = labels_of(adv["C"])
                    C = empty_colmajor([ext[l] for l in lc], device=A.device)
                self.plans.append(Plan.for_tensors(A, la, B, lb, C, lc))
                self.buffers.append(C)
                self.wiring.append((ka, kb))
                work.pop(j)
                work.pop(i)
                work.append((("tmp", s_idx), C, lc))
        except Exception:
            self.close()
            raise

    def execute(self, tensors, stream=None):
        """Runs the steps on the operand tensors (same order, shapes and
        strides as when planned) on `stream` (default: the current stream).
        Returns the result buffer, which the next call overwrites."""
        def get(key):
            return tensors[key[1]] if key[0] == "in" else self.buffers[key[1]]

        for plan, (ka, kb), C in zip(self.plans, self.wiring, self.buffers):
            plan.execute(get(ka), get(kb), C, stream=stream)
        return self.buffers[-1]

    def close(self):
        # the plans' tables must outlive the enqueued steps
        _torch().cuda.synchronize()
        for p in self.plans:
            p.close()
        self.plans = []


def contract_chain(operands, out_labels, order="optimal", out=None):
    """Evaluates the product of the operands ((tensor, labels) pairs, CUDA
    FP64) summed over the labels absent from out_labels.  Returns the result
    (column-major in out_labels order, or written into `out`)."""
    ch = Chain(operands, out_labels, order=order, out=out)
    try:
        return ch.execute([t for t, _ in operands])
    finally:
        ch.close()
