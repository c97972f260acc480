"""GPU parity of tc_execute against the CPU oracle, through the C ABI.

Integer-valued inputs make every partial sum exact, so the GPU must agree
with the oracle bit for bit whatever its summation order; uniform inputs are
held to a componentwise FP64 bound of 1e-12 of (|A||B|)(c)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import FP64_TOL, colmajor_zeros, componentwise_error, reference, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

RECIPES = ["auto", "gemm", "copy_gemm", "gemv", "ger", "dot"]

CASES = [
    # name, labA, labB, labC, extents (sizes span several tiles plus a ragged tail)
    ("3d_matrix", "ikm", "kj", "ijm", {"i": 150, "k": 37, "m": 3, "j": 133}),
    ("cc_a", "abcd", "cdij", "abij", {"a": 12, "b": 11, "c": 9, "d": 7, "i": 6, "j": 5}),
    ("cc_b", "akic", "kbcj", "abij", {"a": 13, "k": 5, "i": 6, "c": 9, "b": 11, "j": 4}),
    ("class31", "abg", "gah", "bh", {"a": 33, "b": 70, "g": 17, "h": 129}),
    ("class32", "abg", "hbg", "ah", {"a": 130, "b": 9, "g": 11, "h": 65}),
    ("xy_b", "iajb", "jgid", "abgd", {"i": 19, "j": 13, "a": 7, "b": 5, "g": 6, "d": 9}),
    ("class2", "abg", "bg", "a", {"a": 300, "b": 17, "g": 9}),
    ("class1", "abg", "abg", "", {"a": 40, "b": 17, "g": 9}),
    ("outer", "ab", "cd", "acbd", {"a": 20, "b": 7, "c": 31, "d": 3}),
    ("batch", "acbdx", "cdx", "abx", {"a": 4, "b": 4, "c": 4, "d": 4, "x": 300}),
    ("c_nonunit_n", "ki", "kj", "ji", {"i": 70, "j": 90, "k": 200}),
    ("long_k", "ik", "kj", "ij", {"i": 65, "j": 66, "k": 3000}),
    ("split_k", "akb", "kbc", "ac", {"a": 31, "k": 600, "b": 37, "c": 5}),   # few tiles, long sum
]


def _run(labA, labB, labC, A, B, recipe, alpha=1.0, beta=0.0, C0=None, tile_id=-1):
    dA, dB = to_dev(A), to_dev(B)
    shape = [dict(zip(labA, A.shape), **dict(zip(labB, B.shape)))[l] for l in labC]
    C = colmajor_zeros(shape)
    if C0 is not None:
        C.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, recipe=recipe, tile_id=tile_id)
    plan.execute(dA, dB, C, alpha, beta)
    torch.cuda.synchronize()
    info = plan.info.as_dict()
    plan.close()
    return C.cpu().numpy(), info


@pytest.mark.parametrize("recipe", RECIPES)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_parity_integer_exact(case, recipe):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(7, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, recipe)
    ref = oracle.contract(A, labA, B, labB, labC)
    print(name, recipe, info["paper_class"], info["recipe_name"], info["M"], info["N"], info["K"], info["L"])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("recipe", RECIPES)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_parity_uniform(case, recipe):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(8, labA, labB, ext, kind="uniform")
    got, info = _run(labA, labB, labC, A, B, recipe)
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print(name, recipe, "componentwise error %.3e" % err)
    assert err <= FP64_TOL


@pytest.mark.parametrize("tile_id", list(range(tc.NUM_TILES)))
def test_every_tile_config(tile_id):
    labA, labB, labC = "akic", "kbcj", "abij"
    ext = {"a": 37, "k": 5, "i": 6, "c": 9, "b": 29, "j": 4}
    A, B = synth.make_operands(9, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "gemm", tile_id=tile_id)
    assert info["tile_id"] == tile_id
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))


def test_alpha_beta_and_nan_output():
    labA, labB, labC, ext = CASES[0][1:]
    A, B = synth.make_operands(10, labA, labB, ext, kind="integers")
    shape = [ext[l] for l in labC]
    C0 = synth.integers(shape, 77)
    got, _ = _run(labA, labB, labC, A, B, "auto", alpha=-0.5, beta=2.0, C0=C0)
    assert np.array_equal(got, -0.5 * oracle.contract(A, labA, B, labB, labC) + 2.0 * C0)
    nan = np.full(shape, np.nan)
    got, _ = _run(labA, labB, labC, A, B, "auto", alpha=1.0, beta=0.0, C0=nan)
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))   # beta = 0 never reads C


def test_strided_views_and_transposed_output():
    g = np.random.default_rng(5)
    big = np.asfortranarray(g.integers(-4, 5, size=(60, 50, 9)).astype(np.float64))
    bigB = np.asfortranarray(g.integers(-4, 5, size=(40, 70)).astype(np.float64))
    A = big[3:53:2, 1:41, ::2]                               # labels i, k, m (non-contiguous)
    B = bigB[:, 5:66]
    dA = to_dev(big)[3:53:2, 1:41, ::2]                      # the same views taken on the device
    dB = to_dev(bigB)[:, 5:66]
    assert not dA.is_contiguous() and dA.stride() == tuple(s // 8 for s in A.strides)
    Ct = torch.zeros(5, 61, 25, dtype=torch.float64, device="cuda").permute(2, 1, 0)   # labels i, j, m
    Cv = Ct.permute(0, 2, 1)                                # i, m, j view of the same storage
    plan = tc.Plan.for_tensors(dA, "ikm", dB, "kj", Cv, "imj")
    plan.execute(dA, dB, Cv)
    torch.cuda.synchronize()
    ref = oracle.contract(A, "ikm", B, "kj", "imj")
    assert np.array_equal(Cv.cpu().numpy(), ref)
    plan.close()


def test_empty_contractions():
    # empty output: no-op
    A = np.zeros((0, 5))
    B = synth.integers((5, 4), 1)
    got, _ = _run("ik", "kj", "ij", A, B, "auto")
    assert got.shape == (0, 4)
    # empty sum: C <- beta * C
    A = np.zeros((3, 0))
    B = np.zeros((0, 4))
    C0 = synth.integers((3, 4), 2)
    got, _ = _run("ik", "kj", "ij", A, B, "auto", beta=3.0, C0=C0)
    assert np.array_equal(got, 3.0 * C0)
    got, _ = _run("ik", "kj", "ij", A, B, "auto", beta=0.0, C0=C0)
    assert not got.any()


def test_random_contractions():
    g = np.random.default_rng(1307)
    for t in range(40):
        la, lb, lc, ext = synth.random_contraction(g, rank_range=(2, 5), ext_range=(2, 12), max_elems=40000,
                                                   p_outer=0.05, allow_batch=True)
        A, B = synth.make_operands(100 + t, la, lb, ext, kind="integers")
        recipe = RECIPES[t % len(RECIPES)]
        got, info = _run(la, lb, lc, A, B, recipe)
        ref = oracle.contract(A, la, B, lb, lc)
        assert np.array_equal(got, ref), (la, lb, lc, ext, recipe, info)


def test_permute_entry_point_bit_exact():
    X = synth.uniform((33, 17, 5, 9), 3)
    for perm in [(1, 0, 2, 3), (3, 2, 1, 0), (0, 2, 1, 3), (2, 3, 0, 1)]:
        ext_out = [X.shape[p] for p in perm]
        st_out = np.cumprod([1] + ext_out[:-1])
        sY = [0] * 4
        for pos, p in enumerate(perm):
            sY[p] = int(st_out[pos])
        dX = to_dev(X)
        Y = torch.zeros(X.size, dtype=torch.float64, device="cuda")
        tc.permute(dX, sY, Y)
        torch.cuda.synchronize()
        assert np.array_equal(Y.cpu().numpy(), oracle.permute(X, sY, X.size)), perm


@pytest.mark.parametrize("case", [
    # class 1 with a long sum: the DOT recipe splits k into segments (second pass)
    ("dot_long", "abc", "abc", "", {"a": 64, "b": 128, "c": 96}),
    # class 2, matrix stride-1 index free (lanes over outputs) and contracted (lanes over k)
    ("gemv_n", "abg", "bg", "a", {"a": 5000, "b": 33, "g": 7}),
    ("gemv_t", "bga", "bg", "a", {"a": 300, "b": 129, "g": 40}),
    ("gemv_few_outputs", "abg", "bg", "a", {"a": 3, "b": 2000, "g": 9}),
    # lanes over outputs with few outputs and a long sum: contracted segments, ordered second pass
    ("gemv_n_segments", "abg", "bg", "a", {"a": 700, "b": 60, "g": 50}),
    # stride-1 modes are different contracted indices: the smaller input is copied first
    ("dot_mismatch", "ij", "ji", "", {"i": 300, "j": 170}),
    ("gemv_t_mismatch", "ijm", "ji", "m", {"i": 70, "j": 90, "m": 33}),
])
def test_memory_bound_recipes(case):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(12, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "auto")
    print(name, info)
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    A, B = synth.make_operands(13, labA, labB, ext, kind="uniform")
    got, info = _run(labA, labB, labC, A, B, "auto", alpha=0.5)
    ref, absr = reference(A, labA, B, labB, labC, alpha=0.5)
    assert componentwise_error(got, ref, absr) <= FP64_TOL


def test_lanes_over_outputs_segments_are_used():
    labA, labB, labC, ext = "abg", "bg", "a", {"a": 700, "b": 60, "g": 50}
    A, B = synth.make_operands(15, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "auto", alpha=2.0, beta=-1.0, C0=synth.integers([700], 3))
    assert info["kernel_name"] == "lanes_over_outputs" and info["workspace_bytes"] > 0, info
    assert np.array_equal(got, 2.0 * oracle.contract(A, labA, B, labB, labC) - synth.integers([700], 3))


def test_split_k_is_used_and_exact():
    labA, labB, labC, ext = "akb", "kbc", "ac", {"a": 31, "k": 600, "b": 37, "c": 5}
    A, B = synth.make_operands(14, labA, labB, ext, kind="integers")
    for recipe in ("auto", "gemm", "copy_gemm"):
        got, info = _run(labA, labB, labC, A, B, recipe)
        assert info["k_split"] > 1, info
        assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))


def test_grid_stride_over_huge_output_counts():
    """DOT recipe forced on a grid contraction with 70M outputs: more
    (output, segment) wavefronts than one grid holds, so the lanes kernel walks
    them grid-stride; sampled outputs against the oracle (bit-exact on integers)."""
    ext = {"a": 4, "b": 4, "c": 4, "d": 4, "x": 1100000}
    labA, labB, labC = "abdx", "dcx", "abcx"
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    dA = torch.randint(-4, 5, [ext[l] for l in reversed(labA)], generator=gen, device="cuda").double().permute(3, 2, 1, 0)
    dB = torch.randint(-4, 5, [ext[l] for l in reversed(labB)], generator=gen, device="cuda").double().permute(2, 1, 0)
    C = colmajor_zeros([ext[l] for l in labC])
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, recipe="dot")
    assert plan.info.kernel == 2 and plan.info.M * plan.info.N * plan.info.L > (1 << 26)
    plan.execute(dA, dB, C)
    torch.cuda.synchronize()
    plan.close()
    g = np.random.default_rng(3)
    idx = np.stack([g.integers(0, ext[l], 400) for l in labC], axis=1)
    idx[:8, 3] = ext["x"] - 1 - np.arange(8)            # include the last points
    s, _ = oracle.contract_entries(dA.cpu().numpy(), labA, dB.cpu().numpy(), labB, labC, idx)
    got = C.cpu().numpy()[tuple(idx.T)]
    assert np.array_equal(got, s)


@pytest.mark.parametrize("case", ["class31", "cc_b", "xy_b", "class32", "3d_matrix"])
def test_suggested_layout_runs_as_direct_gemm(case):
    """Inputs re-stored in the orders tc_suggest_layout proposes plan as one
    direct GEMM with no copy (Class 3.2) and give the oracle's result for the
    original layout."""
    _, la, lb, lc, ext = next(c for c in CASES if c[0] == case)
    A, B = synth.make_operands(11, la, lb, ext, kind="uniform")
    ref, absr = reference(A, la, B, lb, lc)
    out, info = tc.suggest_layout(la, [ext[l] for l in la], lb, [ext[l] for l in lb], lc, [ext[l] for l in lc])
    assert info.paper_class == 32 and info.recipe == tc.TC_RECIPE_GEMM and info.copy_operand == -1

    def restored(X, lab, new):
        return to_dev(np.asfortranarray(np.transpose(X, [lab.index(l) for l in new])))

    dA, dB = restored(A, la, out["A"]), restored(B, lb, out["B"])
    C = colmajor_zeros([ext[l] for l in out["C"]])
    plan = tc.Plan.for_tensors(dA, out["A"], dB, out["B"], C, out["C"])
    try:
        assert plan.info.recipe == tc.TC_RECIPE_GEMM and plan.info.copy_operand == -1
        plan.execute(dA, dB, C)
        torch.cuda.synchronize()
    finally:
        plan.close()
    got = np.transpose(C.cpu().numpy(), [out["C"].index(l) for l in lc])
    err = componentwise_error(got, ref, absr)
    print(case, out, "componentwise error %.3e" % err)
    assert err <= FP64_TOL


@pytest.mark.parametrize("ext,tile,forced", [
    ({"a": 383, "k": 2100, "b": 390}, 1, False),   # the rules: 64x64 tiles + split-K
    ({"a": 777, "k": 2100, "b": 700}, 9, False),   # the rules: 128x128 tiles + split-K
    ({"a": 30, "k": 2100, "b": 600}, 18, False),   # the rules' narrow-column case: 128x32 tiles + split-K,
                                                   # one ragged column tile of 30 < 32
    ({"a": 600, "k": 2100, "b": 30}, 19, False),   # narrow rows: 32x128 tiles + split-K
    ({"a": 40, "k": 2100, "b": 600}, 2, False),    # a column range of 33..48: 128x64 tiles + split-K
    ({"a": 500, "k": 8192, "b": 510}, 11, True),   # split-K on the largest tiles, ragged edges
    ({"a": 380, "k": 8192, "b": 380}, 12, True),
    ({"a": 380, "k": 4096, "b": 380}, 5, True),
    ({"a": 380, "k": 4096, "b": 380}, 2, True),
])
def test_long_contracted_range_tiles_split(ext, tile, forced):
    """Split-K segments and their reduction (one entry per thread, segments
    added in order) on each tile shape: bit-exact on integers."""
    labA, labB, labC = "ak", "kb", "ab"
    A, B = synth.make_operands(15, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "auto", tile_id=tile if forced else -1)
    assert info["tile_id"] == tile and info["k_split"] > 1, info
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
