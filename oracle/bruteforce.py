"""Pure-Python brute-force contraction -- TEST INFRASTRUCTURE ONLY.

For tiny tensors: every combination of index values is visited with
itertools.product and the Einstein sum of the paper (Sec. 2.3, Appendix A:
repeated indices are summed over their whole range) is accumulated in Python
floats.  It pins the C oracle; it is far too slow for anything else.
"""
import itertools

import numpy as np


def contract(A, labA, B, labB, labC):
    labA, labB, labC = list(labA), list(labB), list(labC)
    ext = {}
    for l, e in list(zip(labA, A.shape)) + list(zip(labB, B.shape)):
        if l in ext and ext[l] != e:
            raise ValueError("extent mismatch for label %r" % (l,))
        ext[l] = e
    summed = [l for l in labA if l in labB and l not in labC]
    C = np.zeros([ext[l] for l in labC], dtype=np.float64)
    for cval in itertools.product(*[range(ext[l]) for l in labC]):
        val = dict(zip(labC, cval))
        acc = 0.0
        for sval in itertools.product(*[range(ext[l]) for l in summed]):
            val.update(zip(summed, sval))
            a = float(A[tuple(val[l] for l in labA)])
            b = float(B[tuple(val[l] for l in labB)])
            acc += a * b
        C[cval] = acc
    return C
