"""The GEMM kernel fed by direct global-to-LDS copies (taken for the large
tiles when every operand can be copied in 16-byte pairs along its stride-1
mode), in each of its output tiles (256 x 128, 128 x 256, 192 x 192),
against the oracle: ragged rows, columns and contracted range, k-fast and
row-fast operands in every combination, a free group addressed through an
offset table, contracted groups of several modes (first extent a multiple of
16 or not), a batch index, contracted ranges from one k-tile to several
(the pipelined loop with and without its uniform-offset part), alpha and
beta, and COPY+GEMM feeding it.  Integer inputs must match bit for bit;
uniform inputs are held to the FP64 bound."""
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

CASES = [
    # name, labA, labB, labC, extents: every leading extent even, K not a multiple of 16
    ("cc_a_ragged", "abcd", "cdij", "abij", {"a": 18, "b": 15, "c": 10, "d": 7, "i": 6, "j": 50}),
    ("both_k_fast", "km", "kn", "mn", {"k": 38, "m": 260, "n": 130}),
    ("both_row_fast", "mk", "nk", "mn", {"k": 38, "m": 260, "n": 130}),
    ("table_rows", "kai", "kj", "aji", {"k": 20, "a": 30, "i": 9, "j": 40}),
    ("batch", "kmb", "knb", "mnb", {"k": 36, "m": 260, "n": 130, "b": 3}),
    ("short_k", "km", "kn", "mn", {"k": 2, "m": 300, "n": 140}),
    # contracted groups of two modes (offsets from the digits of k)
    ("cc_b_ragged", "akic", "kbcj", "abij", {"a": 14, "k": 6, "i": 5, "c": 18, "b": 22, "j": 9}),
    ("three_k_modes", "kxmy", "kxny", "mn", {"k": 6, "x": 5, "y": 3, "m": 260, "n": 130}),
    # far fewer rows than one tile
    ("tiny_row_fast", "mk", "nk", "mn", {"k": 34, "m": 2, "n": 4}),
    ("tiny_k_fast", "km", "kn", "mn", {"k": 34, "m": 3, "n": 1}),
    # long contracted ranges: the pipelined loop with uniform tile offsets
    # (first contracted extent a multiple of 16), whole and ragged last tile
    ("long_k_whole", "km", "kn", "mn", {"k": 160, "m": 200, "n": 390}),
    ("long_k_ragged_row_fast", "mk", "kn", "mn", {"k": 150, "m": 394, "n": 198}),
    ("long_k_two_modes", "kxm", "kxn", "mn", {"k": 32, "x": 5, "m": 202, "n": 196}),
    ("long_k_two_modes_ragged", "xkm", "nxk", "mn", {"k": 16, "x": 7, "m": 200, "n": 194}),
]
SHAPES = ["256x128", "128x256", "192x192"]


def _run(labA, labB, labC, A, B, alpha=1.0, beta=0.0, C0=None, shape_name="256x128", recipe="gemm"):
    dA, dB = to_dev(A), to_dev(B)
    shape = [dict(zip(labA, A.shape), **dict(zip(labB, B.shape)))[l] for l in labC]
    C = colmajor_zeros(shape)
    if C0 is not None:
        C.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, recipe=recipe, tile_id=11, copy_tile=shape_name)
    info = plan.info.as_dict()
    plan.execute(dA, dB, C, alpha, beta)
    torch.cuda.synchronize()
    plan.close()
    return C.cpu().numpy(), info


@pytest.mark.parametrize("shape_name", SHAPES)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_copy_fed_gemm_parity(case, shape_name):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(40, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, shape_name=shape_name)
    assert info["copy_fed"] == 1 + tc.COPY_TILES[shape_name] and info["tile_id"] == 11 and info["k_split"] == 1, info
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    A, B = synth.make_operands(41, labA, labB, ext, kind="uniform")
    got, _ = _run(labA, labB, labC, A, B, shape_name=shape_name)
    ref, absr = reference(A, labA, B, labB, labC)
    assert componentwise_error(got, ref, absr) <= FP64_TOL


@pytest.mark.parametrize("shape_name", SHAPES)
def test_copy_fed_alpha_beta(shape_name):
    for name, labA, labB, labC, ext in (CASES[0], CASES[-1]):
        A, B = synth.make_operands(42, labA, labB, ext, kind="integers")
        C0 = synth.integers([ext[l] for l in labC], 43)
        got, info = _run(labA, labB, labC, A, B, alpha=-2.0, beta=0.5, C0=C0, shape_name=shape_name)
        assert info["copy_fed"] == 1 + tc.COPY_TILES[shape_name]
        assert np.array_equal(got, -2.0 * oracle.contract(A, labA, B, labB, labC) + 0.5 * C0)


@pytest.mark.parametrize("shape_name", SHAPES)
def test_copy_gemm_feeds_the_copy_fed_kernel(shape_name):
    """COPY+GEMM on a Class 3.1 contraction: the packed copy of the smaller
    input, then the copy-fed kernel."""
    labA, labB, labC, ext = "abg", "gah", "bh", {"a": 34, "b": 300, "g": 18, "h": 270}
    A, B = synth.make_operands(45, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, shape_name=shape_name, recipe="copy_gemm")
    assert info["copy_operand"] >= 0 and info["copy_fed"] == 1 + tc.COPY_TILES[shape_name], info
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))


def test_odd_leading_extent_keeps_the_gather_kernel():
    labA, labB, labC, ext = "abcd", "cdij", "abij", {"a": 17, "b": 15, "c": 10, "d": 7, "i": 6, "j": 50}
    A, B = synth.make_operands(44, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B)
    assert info["copy_fed"] == 0
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
