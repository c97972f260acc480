"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests retypes the oracle's loop: each compares it with an
independent computation (pure-Python brute force, NumPy routines, the
paper's four slicings of a matrix product, a closed form from Appendix A,
exact rational arithmetic) or checks an invariant that a dropped term, a
wrong index or a transposed operand would break."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SMALL_CASES = [
    # (labA, labB, labC, extents)
    ("ikm", "kj", "ijm", {"i": 3, "k": 4, "m": 2, "j": 5}),          # 3-D x matrix
    ("abcd", "cdij", "abij", {"a": 2, "b": 3, "c": 2, "d": 3, "i": 2, "j": 2}),
    ("akic", "kbcj", "abij", {"a": 3, "k": 2, "i": 2, "c": 3, "b": 2, "j": 2}),
    ("abg", "gah", "bh", {"a": 3, "b": 4, "g": 2, "h": 3}),           # class 3.1
    ("abg", "hbg", "ah", {"a": 3, "b": 4, "g": 2, "h": 3}),           # class 3.2
    ("abg", "abg", "", {"a": 3, "b": 2, "g": 4}),                     # class 1 (scalar)
    ("abg", "bg", "a", {"a": 3, "b": 2, "g": 4}),                     # class 2
    ("ab", "cd", "acbd", {"a": 2, "b": 3, "c": 2, "d": 2}),           # outer product
    ("acbdx", "cdx", "abx", {"a": 2, "b": 3, "c": 2, "d": 2, "x": 3}),  # batch label x
    ("ba", "cb", "ca", {"a": 4, "b": 5, "c": 3}),
]


def _ops(labA, labB, ext, kind, seed):
    A = synth.integers(synth.shape_of(labA, ext), seed) if kind == "int" else \
        synth.uniform(synth.shape_of(labA, ext), seed)
    B = synth.integers(synth.shape_of(labB, ext), seed + 1) if kind == "int" else \
        synth.uniform(synth.shape_of(labB, ext), seed + 1)
    return A, B


@pytest.mark.parametrize("case", SMALL_CASES)
def test_oracle_equals_bruteforce_exactly_on_integers(case):
    labA, labB, labC, ext = case
    A, B = _ops(labA, labB, ext, "int", 11)
    want = bruteforce.contract(A, labA, B, labB, labC)
    for mode in ("plain", "dot2"):
        got = oracle.contract(A, labA, B, labB, labC, mode=mode)
        assert np.array_equal(got, want), mode


@pytest.mark.parametrize("case", SMALL_CASES)
def test_oracle_close_to_bruteforce_on_uniform(case):
    labA, labB, labC, ext = case
    A, B = _ops(labA, labB, ext, "uni", 5)
    want = bruteforce.contract(A, labA, B, labB, labC)
    got = oracle.contract(A, labA, B, labB, labC)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-14)


def test_oracle_handles_strided_views():
    # operands that are non-contiguous views (transposes and steps) of larger arrays
    g = np.random.default_rng(3)
    big = g.integers(-4, 5, size=(7, 6, 5)).astype(np.float64)
    A = big[1:5, ::2, 1:4].transpose(2, 0, 1)    # labels m, i, k
    Bb = g.integers(-4, 5, size=(9, 8)).astype(np.float64)
    B = Bb[::3, 1:6].T                           # labels j, k  (k extent 3 -> need match)
    A = A[:, :, :3]
    want = bruteforce.contract(A, "mik", B, "jk", "ijm")
    got = oracle.contract(A, "mik", B, "jk", "ijm")
    assert np.array_equal(got, want)


def test_matrix_product_four_slicings():
    """Sec. 2.2: C = AB computed from row slices of A (GEMVs), column slices of
    B (GEMVs), a sum of outer products (GERs) and a grid of inner products
    (DOTs) -- all four equal the oracle, exactly on integer data."""
    m, k, n = 6, 5, 7
    A = synth.integers((m, k), 21)
    B = synth.integers((k, n), 22)
    got = oracle.contract(A, "ih", B, "hj", "ij")
    rows = np.stack([A[i, :] @ B for i in range(m)])
    cols = np.stack([A @ B[:, j] for j in range(n)], axis=1)
    ger = sum(np.outer(A[:, h], B[h, :]) for h in range(k))
    dot = np.array([[np.dot(A[i, :], B[:, j]) for j in range(n)] for i in range(m)])
    for ref in (rows, cols, ger, dot, A @ B):
        assert np.array_equal(got, ref)


def test_einsum_cross_check_random_shapes():
    g = np.random.default_rng(7)
    for _ in range(40):
        labA, labB, labC, ext = synth.random_contraction(g, rank_range=(1, 4), ext_range=(1, 5),
                                                         max_elems=400, p_outer=0.1, allow_batch=True)
        A, B = _ops(labA, labB, ext, "uni", int(g.integers(1 << 30)))
        got = oracle.contract(A, labA, B, labB, labC, mode="dot2")
        ref = np.einsum("%s,%s->%s" % (labA, labB, labC), A, B)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13), (labA, labB, labC, ext)


def test_linearity_exact():
    labA, labB, labC, ext = SMALL_CASES[2]
    A1, B = _ops(labA, labB, ext, "int", 31)
    A2, _ = _ops(labA, labB, ext, "int", 41)
    lhs = oracle.contract(2 * A1 + A2, labA, B, labB, labC)
    rhs = 2 * oracle.contract(A1, labA, B, labB, labC) + oracle.contract(A2, labA, B, labB, labC)
    assert np.array_equal(lhs, rhs)


def test_identity_tensor_relabels():
    """Contracting with a Kronecker delta returns the operand with one index renamed."""
    A = synth.uniform((3, 4, 5), 51)
    delta = np.eye(4)
    got = oracle.contract(A, "akc", delta, "kb", "abc")
    assert np.array_equal(got, A)
    delta2 = np.einsum("ik,jl->ikjl", np.eye(3), np.eye(5))  # delta_{ai'} delta_{cj'} as an order-4 tensor
    got2 = oracle.contract(A, "akc", delta2, "apcq", "pkq")
    assert np.array_equal(got2, A)


def test_swap_symmetry():
    """Footnote of Sec. 2.3: with explicit indices the operand order does not matter."""
    for labA, labB, labC, ext in SMALL_CASES:
        A, B = _ops(labA, labB, ext, "int", 61)
        assert np.array_equal(oracle.contract(A, labA, B, labB, labC),
                              oracle.contract(B, labB, A, labA, labC))


def test_storage_permutation_invariance_paper_footnote():
    """Footnote of Sec. 4.1: storing A with its first two indices exchanged and B
    with its first and third exchanged makes R^b_h = A^{abg} B_{gah} compute the
    same R as R^a_h = A^{abg} B_{hbg}."""
    n = 5
    A = synth.integers((n, n, n), 71)
    B = synth.integers((n, n, n), 72)
    R1 = oracle.contract(A, "abg", B, "hbg", "ah")
    At = np.asfortranarray(A.transpose(1, 0, 2))
    Bt = np.asfortranarray(B.transpose(2, 1, 0))
    R2 = oracle.contract(At, "abg", Bt, "gah", "bh")
    assert np.array_equal(R1, R2)
    # and a view with permuted labels is the same tensor: physically permuting
    # storage together with its (extent, stride, label) triples changes nothing
    Ap = np.asfortranarray(A.transpose(2, 0, 1))
    assert np.array_equal(oracle.contract(Ap, "gab", B, "hbg", "ah"), R1)


def test_spherical_metric_closed_form():
    """Appendix A: lowering both indices of S^{mu nu} with g = diag(1, r^2, r^2 sin^2 theta)
    multiplies each entry by the printed power of r and sin(theta)."""
    fx = json.load(open(os.path.join(GOLDEN, "spherical_metric.json")))
    S = synth.uniform((3, 3), 81)
    for r, th in ((2.0, 0.3), (0.5, 1.2), (3.0, 2.5)):
        gdiag = [r ** p * math.sin(th) ** q for p, q in fx["metric_diagonal"]]
        g = np.diag(gdiag)
        T = oracle.contract(g, "am", S, "mn", "an", mode="dot2")     # lower the first index
        low = oracle.contract(T, "an", g, "nb", "ab", mode="dot2")   # then the second
        fac = np.array([[r ** p * math.sin(th) ** q for p, q in row] for row in fx["lowered_factor"]])
        assert np.allclose(low, fac * S, rtol=1e-14, atol=0)


def _gen_ill_dot(n, seed):
    # large products that cancel in pairs (x_i y_i and x_i (-y_i)) hide a sum of
    # small ones: the exact result is O(1) while partial sums reach 2^40
    g = np.random.default_rng(seed)
    m = n // 4
    big = g.uniform(1, 2, m) * 2.0 ** g.integers(30, 40, size=m)
    yb = g.uniform(1, 2, m) * 2.0 ** g.integers(0, 10, size=m)
    xs, ys = g.uniform(-1, 1, n - 2 * m), g.uniform(-1, 1, n - 2 * m)
    x = np.concatenate([big, big, xs])
    y = np.concatenate([yb, -yb, ys])
    perm = g.permutation(n)
    return x[perm], y[perm]


def test_dot2_is_accurate_on_ill_conditioned_sums():
    """The compensated sum is within ~2u of the exact (rational) result where the
    plain sum is far off: the accuracy reference behaves as Dot2 must."""
    u = 2.0 ** -53
    worst_plain = 0.0
    for seed in range(5):
        x, y = _gen_ill_dot(64, seed)
        exact = sum(Fraction(a) * Fraction(b) for a, b in zip(x, y))
        got = oracle.contract(x, "k", y, "k", "", mode="dot2")
        plain = oracle.contract(x, "k", y, "k", "", mode="plain")
        absdot = float(sum(abs(Fraction(a) * Fraction(b)) for a, b in zip(x, y)))
        err = abs(Fraction(float(got)) - exact)
        # Dot2 bound: |res - s| <= u|s| + gamma_{n-1}^2 * sum|x_i y_i|
        gam = (63 * u) / (1 - 63 * u)
        assert err <= u * abs(exact) + 2 * gam * gam * absdot
        worst_plain = max(worst_plain, float(abs(Fraction(float(plain)) - exact) / abs(exact)))
    assert worst_plain > 1e-6   # the cases really are ill conditioned


def test_abs_mode_and_entries_agree_with_full():
    labA, labB, labC, ext = SMALL_CASES[1]
    A, B = _ops(labA, labB, ext, "uni", 91)
    full = oracle.contract(A, labA, B, labB, labC, mode="dot2")
    absf = oracle.contract(np.abs(A), labA, np.abs(B), labB, labC, mode="plain")
    absm = oracle.contract(A, labA, B, labB, labC, mode="abs")
    assert np.allclose(absm, absf, rtol=1e-15, atol=0)
    idx = np.array([[0, 1, 1, 0], [1, 2, 0, 1], [0, 0, 0, 0]])
    s, a = oracle.contract_entries(A, labA, B, labB, labC, idx)
    for e, row in enumerate(idx):
        assert s[e] == full[tuple(row)]
        assert a[e] == absm[tuple(row)]


def test_alpha_beta_semantics():
    labA, labB, labC, ext = SMALL_CASES[0]
    A, B = _ops(labA, labB, ext, "int", 101)
    ref = oracle.contract(A, labA, B, labB, labC)
    C = np.full(ref.shape, np.nan, order="F")
    oracle.contract(A, labA, B, labB, labC, alpha=2.0, beta=0.0, C=C)
    assert np.array_equal(C, 2 * ref)          # beta = 0 never reads C
    C0 = synth.integers(ref.shape, 102)
    C1 = C0.copy(order="F")
    oracle.contract(A, labA, B, labB, labC, alpha=-1.0, beta=3.0, C=C1)
    assert np.array_equal(C1, -ref + 3 * C0)


def test_rejects_non_contractions():
    A = np.zeros((2, 2))
    with pytest.raises(ValueError):
        oracle.contract(A, "aa", A, "ab", "b")      # repeated label within a tensor
    with pytest.raises(ValueError):
        oracle.contract(A, "ab", A, "cd", "ad")     # b summed out of A alone
    with pytest.raises(ValueError):
        oracle.contract(A, "ab", np.zeros((3, 2)), "bc", "ac")  # extent mismatch on b


def test_permute_matches_numpy_transpose():
    X = synth.uniform((3, 4, 5), 111)
    perm = (2, 0, 1)
    Y = np.asfortranarray(X.transpose(perm))
    # strides of X's modes inside Y's column-major storage
    ext_out = [X.shape[p] for p in perm]
    st_out = np.cumprod([1] + ext_out[:-1])
    sY = [0, 0, 0]
    for pos, p in enumerate(perm):
        sY[p] = st_out[pos]
    flat = oracle.permute(X, sY, X.size)
    assert np.array_equal(flat, Y.reshape(-1, order="F"))


def test_empty_extents():
    A = np.zeros((3, 0))
    B = np.zeros((0, 4))
    C = oracle.contract(A, "ik", B, "kj", "ij")
    assert C.shape == (3, 4) and not C.any()      # empty sum is zero
    C2 = oracle.contract(np.zeros((0, 2)), "ik", np.ones((2, 4)), "kj", "ij")
    assert C2.shape == (0, 4)
