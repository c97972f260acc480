"""Oracle for the tensor-contraction library -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU path
computes, written from the paper ("Towards an Efficient Use of the BLAS
Library for Multilinear Tensor Contractions", arXiv:1307.2100).  Only the
tests, the smoke check and the CPU leg of the benchmark may import it; the
library itself never does.

Modules:
  * this file: ctypes front end of the C nested-loop contraction
    (``tc_oracle.c``), plain FP64, compensated Dot2 and |A||B| variants,
    plus the storage permute;
  * ``bruteforce``: pure-Python contraction over every index value, for
    tiny tensors (pins the C oracle);
  * ``slicing``: brute-force enumeration of slicing vectors against the
    requirements R1-R3 and the Delta-classes of Sec. 3 (pins the planner's
    stride classifier);
  * ``mlp_ref``: FP64 forward/backward of the picker's MLP (pins the GPU
    training kernels).
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("TC_ORACLE_LIBRARY") or build_oracle.OUT
        if path == build_oracle.OUT and (not os.path.exists(path) or
                                         os.path.getmtime(path) < os.path.getmtime(build_oracle.SRC)):
            build_oracle.build(force=True)
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.tco_contract.argtypes = ([ctypes.c_int, i64p, i64p, i32p] * 3 +
                                     [dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int])
        lib.tco_contract.restype = ctypes.c_int
        lib.tco_contract_entries.argtypes = ([ctypes.c_int, i64p, i64p, i32p] * 2 +
                                             [ctypes.c_int, i64p, i32p, dp, dp, ctypes.c_int64,
                                              i64p, dp, dp, ctypes.c_int, ctypes.c_int])
        lib.tco_contract_entries.restype = ctypes.c_int
        lib.tco_permute.argtypes = [ctypes.c_int, i64p, i64p, i64p, dp, dp]
        lib.tco_permute.restype = ctypes.c_int
        lib.tco_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


MODES = {"plain": 0, "dot2": 1, "abs": 2}


def labels_of(spec):
    """Labels as int32 codes: a string gives one label per character."""
    if isinstance(spec, str):
        return [ord(ch) for ch in spec]
    return [int(x) for x in spec]


def _i64(seq):
    arr = (ctypes.c_int64 * max(1, len(seq)))()
    for i, v in enumerate(seq):
        arr[i] = int(v)
    return arr


def _i32(seq):
    arr = (ctypes.c_int32 * max(1, len(seq)))()
    for i, v in enumerate(seq):
        arr[i] = int(v)
    return arr


def _elem_strides(x):
    st = []
    for s in x.strides:
        if s % x.itemsize or s < 0:
            raise ValueError("oracle takes non-negative element strides only")
        st.append(s // x.itemsize)
    return st


def _dptr(x):
    return ctypes.cast(ctypes.c_void_p(x.__array_interface__["data"][0]), ctypes.POINTER(ctypes.c_double))


def _desc(x, lab):
    lab = labels_of(lab)
    if x.ndim != len(lab):
        raise ValueError("label count %d != tensor order %d" % (len(lab), x.ndim))
    return [x.ndim, _i64(x.shape), _i64(_elem_strides(x)), _i32(lab)]


def output_extents(A, labA, B, labB, labC):
    la, lb = labels_of(labA), labels_of(labB)
    ext = {}
    for l, e in zip(la, A.shape):
        ext[l] = e
    for l, e in zip(lb, B.shape):
        ext[l] = e
    return tuple(ext[l] for l in labels_of(labC))


def contract(A, labA, B, labB, labC, alpha=1.0, beta=0.0, C=None, mode="plain", nthreads=0):
    """C <- alpha * sum A*B + beta * C (mode "plain" or "dot2"), or the raw
    |A||B| contraction (mode "abs").  A, B, C are FP64 numpy arrays with any
    non-negative strides; a new column-major C is made when C is None."""
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if C is None:
        C = np.zeros(output_extents(A, labA, B, labB, labC), dtype=np.float64, order="F")
        beta = 0.0
    if C.dtype != np.float64:
        raise TypeError("C must be float64")
    args = _desc(A, labA) + _desc(B, labB) + _desc(C, labC)
    rc = lib.tco_contract(*args, _dptr(A), _dptr(B), _dptr(C), float(alpha), float(beta),
                          MODES[mode], int(nthreads))
    if rc:
        raise ValueError("oracle rejected the contraction (code %d)" % rc)
    return C


def contract_entries(A, labA, B, labB, labC, cidx, compensated=True, nthreads=0, with_abs=True):
    """Raw sums sum_k A*B and (with_abs) sum_k |A||B| for selected output entries.

    cidx: (n, rank C) integer array of output multi-indices in labC order."""
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    extC = output_extents(A, labA, B, labB, labC)
    lc = labels_of(labC)
    cidx = np.ascontiguousarray(np.asarray(cidx, dtype=np.int64).reshape(-1, len(lc)))
    n = cidx.shape[0]
    s = np.zeros(n)
    a = np.zeros(n)
    da, db = _desc(A, labA), _desc(B, labB)
    rc = lib.tco_contract_entries(*da, *db, len(lc), _i64(extC), _i32(lc), _dptr(A), _dptr(B), n,
                                  cidx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  _dptr(s), _dptr(a) if with_abs else None, 1 if compensated else 0,
                                  int(nthreads))
    if rc:
        raise ValueError("oracle rejected the contraction (code %d)" % rc)
    return s, a


def permute(X, strides_out, out_size):
    """Y[addrY(idx)] = X[idx] for every multi-index of X; returns flat Y of out_size elements."""
    lib = _load()
    X = np.asarray(X, dtype=np.float64)
    Y = np.zeros(out_size, dtype=np.float64)
    rc = lib.tco_permute(X.ndim, _i64(X.shape), _i64(_elem_strides(X)), _i64(strides_out),
                         _dptr(X), _dptr(Y))
    if rc:
        raise ValueError("oracle permute failed")
    return Y


def max_threads():
    return _load().tco_max_threads()
