"""Host-side tests of the C ABI: the library loads and exports every symbol
include/tc.h declares, the planner's classification agrees with the
brute-force slicing oracle, argument errors come back as status codes, and
the plan's accounting matches the paper's worked numbers.  No GPU needed:
only tc_analyze and the error paths are called."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1307_2100_amd as tc
import synth
from oracle import slicing

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:tc_status|void|const char\s*\*)\s*(tc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    declared = header_functions()
    assert "tc_plan_create" in declared and "tc_execute" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", tc.library_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(tc_\w+)$", out, re.M))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert sorted(tc.EXPORTED) == declared
    assert tc.tc_version() == "1.0.0"


def colmajor_strides(shape):
    st, acc = [], 1
    for e in shape:
        st.append(acc)
        acc *= e
    return st


def desc(labels, ext, strides=None):
    shape = [ext[l] for l in labels]
    return tc.Desc(shape, strides if strides is not None else colmajor_strides(shape), labels)


def analyze(labA, labB, labC, ext, sA=None, sB=None, sC=None, **opt):
    return tc.tc_analyze(desc(labA, ext, sA), desc(labB, ext, sB), desc(labC, ext, sC),
                         tc.make_options(**opt) if opt else None)


def test_paper_class_examples():
    import json
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_slicings.json")))
    for c in fx["classes"]:
        ext = {l: 3 for l in c["T"] + c["S"]}
        info = analyze(c["T"], c["S"], c["R"], ext)
        assert info.paper_class == c["class"], c["where"]


def test_paper_recipes_by_class():
    ext = {l: 4 for l in "abghij"}
    assert analyze("abg", "hbg", "ah", ext).recipe == tc.TC_RECIPE_GEMM          # 3.2
    assert analyze("abg", "gah", "bh", ext).recipe == tc.TC_RECIPE_COPY_GEMM     # 3.1
    assert analyze("abg", "bg", "a", ext).recipe == tc.TC_RECIPE_GEMV            # 2
    assert analyze("abg", "abg", "", ext).recipe == tc.TC_RECIPE_DOT             # 1
    assert analyze("ab", "gh", "abgh", ext).recipe == tc.TC_RECIPE_GER           # outer product
    info = analyze("abg", "gah", "bh", ext, recipe="gemm")
    assert info.recipe == tc.TC_RECIPE_GEMM and info.paper_class == 31


def test_classifier_agrees_with_slicing_oracle_on_random_shapes():
    """The planner's stride-1 rule against brute-force R1-R3 enumeration on
    random contractions with random storage orders (including strided and
    stride-1-free layouts)."""
    g = np.random.default_rng(99)
    seen = set()
    for _ in range(1500):
        la, lb, lc, ext = synth.random_contraction(g, rank_range=(1, 5), ext_range=(2, 4),
                                                   max_elems=10 ** 9, p_outer=0.05, allow_batch=True)
        strides = {}
        units = {}
        for name, labs in (("A", la), ("B", lb)):
            order = list(g.permutation(len(labs)))
            st = [0] * len(labs)
            acc = 1 if g.random() > 0.05 else 2      # sometimes no stride-1 mode at all
            for pos in order:
                st[pos] = acc
                acc *= ext[labs[pos]]
            strides[name] = st
            units[name] = st.index(1) if 1 in st else None
        info = analyze(la, lb, lc, ext, sA=strides["A"], sB=strides["B"])
        want = slicing.classify(la, lb, units["A"], units["B"], lc)
        assert info.paper_class == want, (la, lb, lc, strides)
        seen.add(want)
    assert seen == {0, 1, 2, 31, 32}


def test_table_new3d_through_the_planner():
    ext = {l: 5 for l in "abgh"}
    counts = {31: 0, 32: 0}
    for con in (("b", "g"), ("a", "g"), ("a", "b")):
        free_a = [l for l in "abg" if l not in con][0]
        for order in (con, con[::-1]):
            for pos in (2, 1, 0):
                lb = list(order)
                lb.insert(pos, "h")
                info = analyze("abg", "".join(lb), free_a + "h", ext)
                counts[info.paper_class] += 1
    assert counts == {31: 4, 32: 14}


@pytest.mark.parametrize("bad,status", [
    (("aa", "ab", "b"), "TC_ERR_LABEL"),
    (("ab", "cd", "ad"), "TC_ERR_LABEL"),
    (("ab", "bc", "acd"), "TC_ERR_LABEL"),
])
def test_label_errors(bad, status):
    ext = {l: 3 for l in "abcd"}
    with pytest.raises(tc.TCError) as e:
        analyze(*bad, ext)
    assert tc.STATUS_NAMES[e.value.status] == status
    assert tc.tc_last_error()


def test_extent_overlap_rank_errors():
    with pytest.raises(tc.TCError) as e:
        tc.tc_analyze(tc.Desc([3, 4], [1, 3], "ik"), tc.Desc([5, 2], [1, 5], "kj"), tc.Desc([3, 2], [1, 3], "ij"))
    assert e.value.status == tc.TC_ERR_EXTENT_MISMATCH
    with pytest.raises(tc.TCError) as e:   # C rows and columns share addresses
        tc.tc_analyze(tc.Desc([3, 4], [1, 3], "ik"), tc.Desc([4, 2], [1, 4], "kj"), tc.Desc([3, 2], [1, 2], "ij"))
    assert e.value.status == tc.TC_ERR_OUTPUT_OVERLAP
    with pytest.raises(tc.TCError) as e:
        tc.tc_analyze(tc.Desc([3, 4], [-1, 3], "ik"), tc.Desc([4, 2], [1, 4], "kj"), tc.Desc([3, 2], [1, 3], "ij"))
    assert e.value.status == tc.TC_ERR_INVALID_ARG
    big = "abcdefghijklmnopq"
    with pytest.raises(tc.TCError) as e:
        tc.tc_analyze(tc.Desc([1] * 17, [1] * 17, big), tc.Desc([1], [1], "a"), tc.Desc([1] * 16, [1] * 16, big[1:]))
    assert e.value.status == tc.TC_ERR_RANK
    with pytest.raises(tc.TCError) as e:
        analyze("ik", "kj", "ij", {"i": 2, "k": 2, "j": 2}, recipe=9)
    assert e.value.status == tc.TC_ERR_INVALID_ARG
    # every enum field is checked as a plain int at the ABI (a C caller may store
    # any value there; reading it as the enum type first would be undefined)
    for bad in (dict(precision=4), dict(precision=-1), dict(recipe=-3), dict(picker=3), dict(picker=1 << 20)):
        with pytest.raises(tc.TCError) as e:
            analyze("ik", "kj", "ij", {"i": 2, "k": 2, "j": 2}, **bad)
        assert e.value.status == tc.TC_ERR_INVALID_ARG, bad


def test_execute_rejects_null_plan_and_small_workspace_without_gpu():
    with pytest.raises(tc.TCError) as e:
        tc.tc_execute(None, None, None, None, 1.0, 0.0, None, 0, None)
    assert e.value.status == tc.TC_ERR_INVALID_ARG


def test_group_sizes_fusion_and_flops():
    labA, labB, labC, ext = synth.workload_cc_a(128, 32)
    info = analyze(labA, labB, labC, ext)
    # C's stride-1 index a is free in A, so the kernel takes B as its A
    assert info.swapped == 1
    assert (info.M, info.N, info.K, info.L) == (32 * 32, 128 * 128, 128 * 128, 1)
    assert (info.nM, info.nN, info.nK) == (1, 1, 1)      # every group fuses to one mode
    assert info.flops == 549755813888.0
    assert info.bytes == 8 * (128 ** 4 + 2 * 128 ** 2 * 32 ** 2)
    labA, labB, labC, ext = synth.workload_cc_b(128, 32)
    info = analyze(labA, labB, labC, ext)
    assert info.paper_class == 32 and info.recipe == tc.TC_RECIPE_GEMM
    assert (info.nM, info.nN, info.nK) == (2, 2, 2)      # (b,j), (a,i), (k,c) do not fuse
    assert info.flops == 137438953472.0


def test_equal_operation_counts_paper_footnotes():
    """Sec. 4.1 footnote: the two 3-D contractions do the same arithmetic;
    Sec. 4.2 footnote: so do the two coupled-cluster ones."""
    ext = {l: 7 for l in "abgh"}
    assert analyze("abg", "hbg", "ah", ext).flops == analyze("abg", "gah", "bh", ext).flops
    ext = {"i": 9, "j": 9, "a": 3, "b": 4, "g": 5, "d": 6}
    assert analyze("iajb", "igjd", "abgd", ext).flops == analyze("iajb", "jgid", "abgd", ext).flops


def test_memory_size_worked_example():
    """Sec. 4.2: X^{i a j b} with a = b = 80 and i = j = 2000 takes 204 GB in FP64."""
    ext = {"i": 2000, "j": 2000, "a": 80, "b": 80, "g": 80, "d": 80}
    info = analyze("iajb", "igjd", "abgd", ext)
    x_bytes = 8 * 2000 * 2000 * 80 * 80
    assert x_bytes == 204_800_000_000
    assert info.bytes == 2 * x_bytes + 8 * 80 ** 4


def test_copy_recipe_workspace_and_operand():
    ext = {l: 6 for l in "abgh"}
    info = analyze("abg", "gah", "bh", ext)
    assert info.recipe == tc.TC_RECIPE_COPY_GEMM
    assert info.workspace_bytes == 8 * 6 ** 3 and info.copy_operand in (0, 1)
    ext2 = dict(ext, h=3)        # B smaller: B is copied
    assert analyze("abg", "gah", "bh", ext2).copy_operand == 1


def test_inner_products_copy_when_stride1_modes_are_different_contracted_indices():
    # DOT of A[i,j] and B[j,i]: the stride-1 modes i and j are both contracted
    # and differ (Class 3.1's failure F1 for a BLAS-1 slice): the smaller
    # input is copied into the other's contracted order first
    info = analyze("ij", "ji", "", {"i": 40, "j": 30})
    assert info.recipe == tc.TC_RECIPE_DOT and info.copy_operand in (0, 1)
    assert info.workspace_bytes >= 8 * 40 * 30
    # same order: no copy
    assert analyze("ij", "ij", "", {"i": 40, "j": 30}).copy_operand == -1
    # GEMV with the vector in another contracted order: the vector is copied
    info = analyze("ijm", "ji", "m", {"i": 20, "j": 30, "m": 50})
    assert info.recipe == tc.TC_RECIPE_GEMV and info.copy_operand >= 0
    # the vector's stride-1 mode is the matrix's: no copy
    assert analyze("ijm", "ij", "m", {"i": 20, "j": 30, "m": 50}).copy_operand == -1


def test_empty_and_degenerate_shapes_analyze():
    info = analyze("ik", "kj", "ij", {"i": 0, "k": 3, "j": 2})
    assert info.M == 0 and info.flops == 0
    info = analyze("ik", "kj", "ij", {"i": 4, "k": 0, "j": 2})
    assert info.K == 0
    info = analyze("ik", "kj", "ij", {"i": 1, "k": 1, "j": 1})
    assert (info.M, info.N, info.K) == (1, 1, 1)


def test_single_hip_runtime_in_process():
    """libtc must share PyTorch's HIP runtime: two runtimes in one process do
    not see the same device."""
    maps = open("/proc/self/maps").read()
    libs = set(l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l)
    assert len(libs) == 1, libs


def test_split_precision_plans_have_no_copy_step():
    """Split precision gathers both inputs into digit planes itself: even a
    Class 3.1 contraction gets no COPY step (its operand strides must stay the
    caller's)."""
    ext = {l: 6 for l in "abgh"}
    info = analyze("abg", "gah", "bh", ext, precision="split_bf16")
    assert info.paper_class == 31 and info.copy_operand == -1 and info.split_slices == 5
    assert info.workspace_bytes > 0
    info = analyze("abg", "gah", "bh", ext, precision="split_fp8")
    assert info.split_slices == 8


CRT_MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199]


def test_crt_moduli_are_pairwise_coprime_and_fit_int8():
    """Residues in [-floor(p/2), ceil(p/2) - 1] must fit in int8 and the
    moduli must be pairwise coprime for the Chinese remainder theorem."""
    import math
    for i, p in enumerate(CRT_MODULI):
        assert -(p // 2) >= -128 and (p + 1) // 2 - 1 <= 127
        for q in CRT_MODULI[i + 1:]:
            assert math.gcd(p, q) == 1, (p, q)


def test_crt_plan_bits_and_limits():
    """The residue form keeps b bits per input, the largest b <= 48 with
    2 K 4^b < P (P the product of the moduli used), so that every sum of K
    products of integers |a|, |b| <= 2^b is recovered without ambiguity."""
    def expected_bits(n, K):
        P = 1
        for p in CRT_MODULI[:n]:
            P *= p
        return max([b for b in range(1, 49) if 2 * K * 4 ** b < P] or [0])

    def default_moduli(K):
        return min([n for n in range(2, 15) if expected_bits(n, K) >= 40] or [14])

    ext = {"i": 40, "k": 300, "j": 7}
    info = analyze("ik", "kj", "ij", ext, precision="crt_int8")
    assert info.split_slices == default_moduli(300) == 12 and info.split_bits == expected_bits(12, 300) >= 40
    for K in (2, 300, 4096, 16384, 36864, 1 << 20, 1 << 24):
        i = analyze("ik", "kj", "ij", {"i": 3, "k": K, "j": 2}, precision="crt_int8")
        assert i.split_slices == default_moduli(K) and i.split_bits == expected_bits(i.split_slices, K)
    assert info.kernel == 4 and info.workspace_bytes > 0 and info.precision == tc.TC_PREC_F64_CRT_INT8
    for n in range(2, 15):
        for K in (1, 4, 300, 4096, 36864, 70000):
            e = {"i": 3, "k": K, "j": 2}
            b = expected_bits(n, K)
            if b == 0:
                with pytest.raises(tc.TCError) as err:
                    analyze("ik", "kj", "ij", e, precision="crt_int8", split_slices=n)
                assert err.value.status == tc.TC_ERR_UNSUPPORTED
            else:
                assert analyze("ik", "kj", "ij", e, precision="crt_int8", split_slices=n).split_bits == b
    for n in (1, 15):
        with pytest.raises(tc.TCError) as err:
            analyze("ik", "kj", "ij", ext, precision="crt_int8", split_slices=n)
        assert err.value.status == tc.TC_ERR_INVALID_ARG
    # residue GEMM configurations: tile_id picks one, -1 the default, others are rejected
    assert analyze("ik", "kj", "ij", ext, precision="crt_int8", tile_id=2).tile_id == 2
    assert 0 <= info.tile_id < tc.CRT_NUM_TILES
    with pytest.raises(tc.TCError) as err:
        analyze("ik", "kj", "ij", ext, precision="crt_int8", tile_id=tc.CRT_NUM_TILES)
    assert err.value.status == tc.TC_ERR_INVALID_ARG
    header = open(HEADER).read()
    assert re.search(r"#define TC_CRT_NUM_TILES %d\b" % tc.CRT_NUM_TILES, header)
    # the digit forms report their bits too: 8 + 9 (S - 1) for BF16, 4 + 5 (S - 1) for FP8
    assert analyze("ik", "kj", "ij", ext, precision="split_bf16").split_bits == 44
    assert analyze("ik", "kj", "ij", ext, precision="split_fp8").split_bits == 39
    assert analyze("ik", "kj", "ij", ext).split_bits == 0


def test_copy_fed_gemm_eligibility():
    """The copy-fed FP64 kernel is planned for the large tiles (256x128 and
    128x256, no split-K; also after the copy of COPY+GEMM) when every operand's
    stride-1 mode leads its row or contracted group with an even extent and
    every other stride is even."""
    for la, lb, lc, ext in (synth.workload_cc_a(128, 32), synth.workload_cc_b(128, 32)):
        info = analyze(la, lb, lc, ext)
        assert info.tile_id == 11 and info.k_split == 1 and info.copy_fed == 1
    ext = {"a": 18, "b": 15, "c": 10, "d": 7, "i": 6, "j": 50}
    assert analyze("abcd", "cdij", "abij", ext, recipe="gemm", tile_id=11).copy_fed == 1
    assert analyze("abcd", "cdij", "abij", ext, recipe="gemm", tile_id=12).copy_fed == 2
    assert analyze("abcd", "cdij", "abij", ext, recipe="gemm", tile_id=0).copy_fed == 0       # other tile
    assert analyze("abcd", "cdij", "abij", ext, recipe="copy_gemm", tile_id=11).copy_fed == 1  # after the COPY step
    assert analyze("abcd", "cdij", "abij", ext, precision="crt_int8").copy_fed == 0
    odd = dict(ext, a=17)                                       # odd leading extent of the row-fast operand
    assert analyze("abcd", "cdij", "abij", odd, recipe="gemm", tile_id=11).copy_fed == 0
    oddk = dict(ext, c=9)                                       # odd leading extent of the k-fast operand
    assert analyze("abcd", "cdij", "abij", oddk, recipe="gemm", tile_id=11).copy_fed == 0
    # a strided (every other entry) view keeps no stride-1 mode: no 16-byte pairs
    sA = colmajor_strides([18, 15, 10, 7])
    assert analyze("abcd", "cdij", "abij", ext, sA=[2 * x for x in sA], recipe="gemm", tile_id=11).copy_fed == 0
    # an explicit copy-fed tile overrides the tile's own shape
    for name, code in tc.COPY_TILES.items():
        assert analyze("abcd", "cdij", "abij", ext, recipe="gemm", tile_id=11, copy_tile=name).copy_fed == 1 + code
    with pytest.raises(tc.TCError):
        analyze("abcd", "cdij", "abij", ext, copy_tile=3)


def test_copy_fed_tile_rule():
    """Without a tile asked for, the copy-fed kernel takes the output tile
    whose workgroups (one per compute unit of 256, dealt out in rounds) leave
    the least output area in flight: the v=192, o=48 coupled-cluster shapes
    (2304 x 36864 and 9216 x 9216 outputs) divide into exactly 9 rounds of
    192 x 192 tiles, against 10.1 rounds of 256 x 128; the v=128, o=32 ones
    (1024 x 16384, 4096 x 4096) into 2 rounds of 256 x 128."""
    def rounds_area(M, N, bm, bn):
        tiles = -(-M // bm) * -(-N // bn)
        return -(-tiles // 256) * bm * bn

    for (la, lb, lc, ext), want in ((synth.workload_cc_a(192, 48), 3), (synth.workload_cc_b(192, 48), 3),
                                     (synth.workload_cc_a(128, 32), 1), (synth.workload_cc_b(128, 32), 1)):
        info = analyze(la, lb, lc, ext)
        assert info.copy_fed == want, (ext, info.copy_fed)
        costs = [rounds_area(info.M, info.N, bm, bn) for bm, bn in ((256, 128), (128, 256), (192, 192))]
        assert info.copy_fed == 1 + int(np.argmin(costs))
    # a tile asked for keeps its own shape
    la, lb, lc, ext = synth.workload_cc_a(192, 48)
    assert analyze(la, lb, lc, ext, recipe="gemm", tile_id=11).copy_fed == 1


def test_fast_division_method():
    """The slab engine divides by plan-time constants with a multiply and a
    shift (mul = ceil(2^p / d), p = 31 + ceil(log2 d)); check the method
    against exact integer division on 0 <= n < 2^31."""
    g = np.random.default_rng(17)
    divisors = list(range(1, 3000)) + [int(x) for x in g.integers(3000, 1 << 30, 300)] + [(1 << 30) + 1, (1 << 31) - 1]
    for d in divisors:
        if d == 1:
            continue
        l = (d - 1).bit_length()
        p = 31 + l
        mul = ((1 << p) + d - 1) // d
        assert mul < (1 << 32)
        ns = [0, 1, d - 1, d, d + 1, (1 << 31) - 1, (1 << 31) - 2] + [int(x) for x in g.integers(0, 1 << 31, 50)]
        for n in ns:
            assert ((n * mul) >> 32) >> (p - 32) == n // d, (n, d)


def test_long_contracted_range_tile_rule():
    """Few output tiles over a long contracted range: the rules take 128x32
    tiles for a column range of at most 32 beside a long row range (32x128
    for a row range of at most 32), 128x64 tiles for a column range of at
    most 48, else
    128x128 tiles, else 64x64, when padding wastes under a quarter of the tile and
    split-K turns them into 256 or more workgroups; failing that they still
    move from 32x32 tiles (no split-K at 128 tiles or more) to 64x64 or
    128x128 tiles that split the range."""
    for (m, k, n), tile in (((384, 147456, 384), 9), ((512, 262144, 512), 9), ((192, 36864, 192), 1),
                            ((3600, 10 ** 6, 60), 1), ((2025, 10 ** 6, 45), 1), ((1000, 3000, 1000), 9),
                            ((256, 10000, 256), 1), ((383, 2100, 390), 1), ((777, 2100, 700), 9),
                            ((30, 10 ** 6, 900), 18), ((900, 10 ** 6, 30), 19), ((45, 10 ** 6, 2025), 2),
                            ((33, 10 ** 6, 900), 2)):
        info = analyze("ak", "kb", "ab", {"a": m, "k": k, "b": n})
        assert info.tile_id == tile and info.k_split > 1, (m, k, n, info.tile_id)
    # short range or enough tiles: unchanged
    assert analyze("ak", "kb", "ab", {"a": 383, "k": 1000, "b": 390}).tile_id == 8
    assert analyze("ak", "kb", "ab", {"a": 100, "k": 100000, "b": 100}).tile_id == 8
    assert analyze("ak", "kb", "ab", {"a": 4096, "k": 4096, "b": 4096}).tile_id == 11


# ------------------------------------------------------------------ sizes
# Every size the planner forms is a product of extents.  Layouts whose element
# counts, address spans or iteration space pass 2^56 are rejected with a
# status code before any product can wrap (zero strides make such extents
# reachable without the memory to hold them).
BIG = 1 << 20


def _status_of(fn):
    with pytest.raises(tc.TCError) as e:
        fn()
    return e.value.status


def test_overflowing_extent_products_are_rejected_not_wrapped():
    # four modes of 2^20 with strides 1, 2^20, 2^40, 2^60: the element count is 2^80
    huge = tc.Desc([BIG] * 4, [1, BIG, 1 << 40, 1 << 60], "abcd")
    B = tc.Desc([BIG] * 4, [1, BIG, 1 << 40, 1 << 60], "cdef")
    C = tc.Desc([BIG] * 4, [1, BIG, 1 << 40, 1 << 60], "abef")
    st = _status_of(lambda: tc.tc_analyze(huge, B, C))
    assert st == tc.TC_ERR_INVALID_ARG
    assert "2^56" in tc.tc_last_error()
    # the same extents as a full contraction to a scalar: K = 2^80 used to wrap to 0
    B2 = tc.Desc([BIG] * 4, [1, BIG, 1 << 40, 1 << 60], "abcd")
    st = _status_of(lambda: tc.tc_analyze(huge, B2, tc.Desc([], [], "")))
    assert st == tc.TC_ERR_INVALID_ARG


def test_zero_stride_inputs_with_a_huge_iteration_space_are_rejected():
    # broadcast inputs (stride 0 along k) of 2^48 entries each, and an output
    # of 2^40: each tensor fits, but the contraction has 2^68 terms
    A = tc.Desc([1 << 28, 1 << 20], [0, 1], "ki")
    B = tc.Desc([1 << 28, 1 << 20], [0, 1], "kj")
    C = tc.Desc([1 << 20, 1 << 20], [1, 1 << 20], "ij")
    st = _status_of(lambda: tc.tc_analyze(A, B, C))
    assert st == tc.TC_ERR_INVALID_ARG
    assert "iteration space" in tc.tc_last_error()


def test_address_span_overflow_is_rejected():
    # 3 entries 2^62 apart: the span, not the count, leaves int64
    A = tc.Desc([3, 2], [1 << 62, 1], "ka")
    B = tc.Desc([3], [1], "k")
    C = tc.Desc([2], [1], "a")
    assert _status_of(lambda: tc.tc_analyze(A, B, C)) == tc.TC_ERR_INVALID_ARG
    assert "span" in tc.tc_last_error()


def test_sizes_at_the_limit_still_plan():
    # iteration space exactly 2^56 through broadcast (stride-0) inputs, no overflow anywhere
    A = tc.Desc([1 << 28, 1 << 14], [0, 1], "ki")
    B = tc.Desc([1 << 28, 1 << 14], [0, 1], "kj")
    C = tc.Desc([1 << 14, 1 << 14], [1, 1 << 14], "ij")
    info = tc.tc_analyze(A, B, C)
    assert (info.M, info.N, info.K) == (1 << 14, 1 << 14, 1 << 28)
    assert info.flops == 2.0 * 2 ** 56
    # one factor of two more is rejected
    A2 = tc.Desc([1 << 29, 1 << 14], [0, 1], "ki")
    B2 = tc.Desc([1 << 29, 1 << 14], [0, 1], "kj")
    assert _status_of(lambda: tc.tc_analyze(A2, B2, C)) == tc.TC_ERR_INVALID_ARG
    # the split-precision workspace of a near-limit plan is a checked sum, not a wrapped one
    for prec in ("split_bf16", "split_fp8", "crt_int8"):
        try:
            info = tc.tc_analyze(A, B, C, tc.make_options(precision=prec))
            assert info.workspace_bytes > 2 * (1 << 42)   # the planes hold every input digit
        except tc.TCError as e:
            assert e.status in (tc.TC_ERR_INVALID_ARG, tc.TC_ERR_UNSUPPORTED)


def test_unfusable_groups_beyond_the_table_cap_are_unsupported():
    # a two-mode free group that does not fuse (C stores it transposed) needs
    # one offset-table entry per index; 2^32 entries exceed the cap
    A = tc.Desc([1 << 16, 1 << 16, 2], [1, 0, 0], "abk")
    B = tc.Desc([2, 3], [1, 2], "kj")
    C = tc.Desc([1 << 16, 1 << 16, 3], [1 << 16, 1, 1 << 32], "abj")
    assert _status_of(lambda: tc.tc_analyze(A, B, C)) == tc.TC_ERR_UNSUPPORTED
    assert "offset-table" in tc.tc_last_error()


def test_permute_rejects_overflowing_sizes_without_gpu():
    st = _status_of(lambda: tc.tc_permute([BIG] * 4, [1, BIG, 1 << 40, 1 << 60], [1, BIG, 1 << 40, 1 << 60],
                                          None, None, None))
    assert st == tc.TC_ERR_INVALID_ARG
