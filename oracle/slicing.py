"""Brute-force slicing analysis -- TEST INFRASTRUCTURE ONLY.

Written from Sec. 2.4 and Sec. 3 of the paper.  A slicing is a pair of 0/1
vectors s(T), s(S) (1 = the mode is sliced, i.e. looped over; Sec. 2.4).
Slicing a contracted index slices it in both operands (remark under R2), so
the two vectors agree on every contracted label.  Every such pair is
enumerated and tested against

  R1  the stride-1 modes of T and S are not sliced,
  R2  |s(T)|_1 = N(T)-2 and |s(S)|_1 = N(S)-2,
  R3  each slice keeps exactly one free and one contracted index,

and the BLAS kernel that the slices feed is read off what stays unsliced
(Sec. 2.2 for the matrix case: two matrices -> GEMM, a matrix and a vector
-> GEMV, two vectors sharing the contracted index -> DOT, two vectors with
no contracted index -> GER; Sec. 3.1 F1: a matrix slice that lost its
stride-1 mode needs a copy first).

The classes come from Sec. 3.2: Delta(t) = N(t) - p; Class 1 when both are 0,
Class 2 when exactly one is 0, Class 3 when both are >= 1.  Class 3 is split
constructively here: 3.2 when some slicing satisfies R1, R2 and R3 (GEMM
directly), 3.1 when only R2 and R3 can be met (COPY+GEMM).  The library's
classifier uses the paper's stride-1 rule instead; the tests check that the
two agree.

Readings where the paper is silent: labels present in T, S and the output
(batch labels) are sliced in all operands and not counted in N(t); a tensor
with no stride-1 mode cannot satisfy R1; p = 0 is an outer product (class 0).
"""
import itertools


def kernel_of(fT, fS, c, unit_kept_T, unit_kept_S):
    """BLAS kernel fed by slices keeping fT free modes of T, fS of S and c
    shared contracted modes unsliced."""
    if (fT, fS, c) == (1, 1, 1):
        return "GEMM" if (unit_kept_T and unit_kept_S) else "COPY+GEMM"
    if (fT, fS, c) == (1, 0, 1):
        return "GEMV" if unit_kept_T else "COPY+GEMV"
    if (fT, fS, c) == (0, 1, 1):
        return "GEMV" if unit_kept_S else "COPY+GEMV"
    if fT == 0 and fS == 0 and c >= 1:
        # only contracted modes left: an inner product over them (the third
        # choice for example (1') of Sec. 3.2 keeps two and calls it DOT)
        return "DOT"
    if (fT, fS, c) == (1, 1, 0):
        return "GER"
    if (fT, fS, c) in ((1, 0, 0), (0, 1, 0)):
        return "AXPY"
    if (fT, fS, c) == (0, 0, 0):
        return "SCALAR"
    return None


def enumerate_slicings(labT, labS, unitT, unitS, labR=None):
    """Yield dicts describing every consistent slicing of T and S.

    labT, labS: labels in storage order.  unitT, unitS: position of the
    stride-1 mode (None if the tensor has none).  labR: output labels; when
    given, labels in all three tensors are batch labels (always sliced).
    """
    labT, labS = list(labT), list(labS)
    batch = set()
    if labR is not None:
        batch = set(labT) & set(labS) & set(labR)
    contracted = [l for l in labT if l in labS and l not in batch]
    NT = len(labT) - len([l for l in labT if l in batch])
    NS = len(labS) - len([l for l in labS if l in batch])
    freeT = [l for l in labT if l not in labS]
    freeS = [l for l in labS if l not in labT]
    for sc in itertools.product((0, 1), repeat=len(contracted)):
        cs = dict(zip(contracted, sc))
        for sft in itertools.product((0, 1), repeat=len(freeT)):
            fts = dict(zip(freeT, sft))
            for sfs in itertools.product((0, 1), repeat=len(freeS)):
                fss = dict(zip(freeS, sfs))
                sT = []
                for l in labT:
                    sT.append(1 if l in batch else cs.get(l, fts.get(l)))
                sS = []
                for l in labS:
                    sS.append(1 if l in batch else cs.get(l, fss.get(l)))
                kept_f_T = sum(1 for l in freeT if fts[l] == 0)
                kept_f_S = sum(1 for l in freeS if fss[l] == 0)
                kept_c = sum(1 for l in contracted if cs[l] == 0)
                keptT_unit = unitT is not None and sT[unitT] == 0
                keptS_unit = unitS is not None and sS[unitS] == 0
                nsT = sum(sT) - sum(1 for l in labT if l in batch)
                nsS = sum(sS) - sum(1 for l in labS if l in batch)
                r1 = keptT_unit and keptS_unit
                r2 = nsT == NT - 2 and nsS == NS - 2
                r3 = kept_f_T == 1 and kept_f_S == 1 and kept_c == 1
                yield {
                    "sT": tuple(sT), "sS": tuple(sS),
                    "R1": r1, "R2": r2, "R3": r3,
                    "kernel": kernel_of(kept_f_T, kept_f_S, kept_c, keptT_unit, keptS_unit),
                    "unsliced": tuple(l for l, s in zip(labT, sT) if s == 0)
                    + tuple(l for l, s in zip(labS, sS) if s == 0 and l not in labT),
                }


def delta(labT, labS, labR=None):
    """(Delta(T), Delta(S), p): free-index counts and number of contractions."""
    batch = set(labT) & set(labS) & set(labR) if labR is not None else set()
    p = len([l for l in labT if l in labS and l not in batch])
    NT = len([l for l in labT if l not in batch])
    NS = len([l for l in labS if l not in batch])
    return NT - p, NS - p, p


def classify(labT, labS, unitT, unitS, labR=None):
    """Paper class as 0 (outer product, p = 0), 1, 2, 31 or 32."""
    dT, dS, p = delta(labT, labS, labR)
    if p == 0:
        return 0
    if dT == 0 and dS == 0:
        return 1
    if dT == 0 or dS == 0:
        return 2
    slicings = list(enumerate_slicings(labT, labS, unitT, unitS, labR))
    if any(s["R1"] and s["R2"] and s["R3"] for s in slicings):
        return 32
    if any(s["R2"] and s["R3"] for s in slicings):
        return 31
    raise AssertionError("class 3 contraction without an R2/R3 slicing")


def gemm_slicings(labT, labS, unitT, unitS, labR=None):
    """All slicings that satisfy R1, R2 and R3 (direct GEMM)."""
    return [s for s in enumerate_slicings(labT, labS, unitT, unitS, labR)
            if s["R1"] and s["R2"] and s["R3"]]
