"""Split-precision contractions (FP64 digits on BF16 / FP8 matrix cores, and
FP64 inputs as integers multiplied through INT8 residues) against the
compensated FP64 oracle.

Integer-valued inputs in [-4, 4] fit in one digit, and in the integer form
of the residue path, so every product and sum is exact and the result must
equal the oracle bit for bit.  Otherwise the componentwise error must stay
within the bound of the bits kept per input: BF16 with the default 5 digits
(8 + 4x9 = 44 bits) and the residue form with its default moduli (at least
40 bits) are held to 1e-10, also on inputs whose slices are scaled by
10^U(-3,3)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import colmajor_zeros, componentwise_error, reference, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

SPLIT_TOL = 1e-10

CASES = [
    ("3d_matrix", "ikm", "kj", "ijm", {"i": 150, "k": 300, "m": 3, "j": 133}),
    ("cc_a", "abcd", "cdij", "abij", {"a": 12, "b": 11, "c": 19, "d": 17, "i": 6, "j": 5}),
    ("cc_b", "akic", "kbcj", "abij", {"a": 13, "k": 5, "i": 6, "c": 39, "b": 11, "j": 4}),
    ("class31", "abg", "gah", "bh", {"a": 33, "b": 70, "g": 17, "h": 129}),
    ("class2", "abg", "bg", "a", {"a": 300, "b": 17, "g": 9}),
]


def _run(labA, labB, labC, A, B, precision, slices=0, alpha=1.0, beta=0.0, C0=None, tile=-1):
    dA, dB = to_dev(A), to_dev(B)
    shape = [dict(zip(labA, A.shape), **dict(zip(labB, B.shape)))[l] for l in labC]
    C = colmajor_zeros(shape)
    if C0 is not None:
        C.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, precision=precision, split_slices=slices, tile_id=tile)
    plan.execute(dA, dB, C, alpha, beta)
    torch.cuda.synchronize()
    info = plan.info.as_dict()
    plan.close()
    return C.cpu().numpy(), info


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp8", "crt_int8"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_exact_on_integers(case, precision):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(21, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, precision)
    assert info["split_slices"] > 0 and info["precision"] == tc.PRECISIONS[precision]
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))


@pytest.mark.parametrize("kind", ["uniform", "scaled_normal"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_bf16_default_meets_1e10(case, kind):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(22, labA, labB, ext, kind=kind)
    got, info = _run(labA, labB, labC, A, B, "split_bf16")
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print(name, kind, "bf16 S=%d componentwise error %.3e" % (info["split_slices"], err))
    assert err <= SPLIT_TOL


@pytest.mark.parametrize("kind", ["uniform", "scaled_normal"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_crt_default_meets_1e10(case, kind):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(25, labA, labB, ext, kind=kind)
    got, info = _run(labA, labB, labC, A, B, "crt_int8")
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print(name, kind, "crt %d moduli, %d bits: componentwise error %.3e" % (info["split_slices"], info["split_bits"], err))
    assert info["split_bits"] >= 40
    assert err <= SPLIT_TOL


@pytest.mark.parametrize("tile", range(tc.CRT_NUM_TILES))
def test_crt_every_gemm_configuration(tile):
    """Every residue GEMM configuration (register-staged and LDS-ring) on a
    shape with ragged rows, columns and a contracted range of several
    k-steps: exact on integers, within the bound on real inputs."""
    labA, labB, labC = "ikm", "kj", "ijm"
    ext = {"i": 150, "k": 300, "m": 3, "j": 301}
    A, B = synth.make_operands(30, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "crt_int8", tile=tile)
    assert info["tile_id"] == tile
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    A, B = synth.make_operands(31, labA, labB, ext, kind="uniform")
    got, info = _run(labA, labB, labC, A, B, "crt_int8", tile=tile)
    ref, absr = reference(A, labA, B, labB, labC)
    assert componentwise_error(got, ref, absr) <= SPLIT_TOL


def test_crt_error_falls_with_moduli():
    """Rounding each input to b bits below its row scale errs by at most
    2^-(b+1) of that scale per entry; more moduli buy more bits (about 4 per
    modulus) until FP64 rounding of the result dominates."""
    name, labA, labB, labC, ext = CASES[1]
    A, B = synth.make_operands(26, labA, labB, ext, kind="scaled_normal")
    ref, absr = reference(A, labA, B, labB, labC)
    errs, bits = [], []
    for n in range(2, 15):
        got, info = _run(labA, labB, labC, A, B, "crt_int8", slices=n)
        errs.append(componentwise_error(got, ref, absr))
        bits.append(info["split_bits"])
    print("crt", list(zip(bits, ["%.2e" % e for e in errs])))
    for b, e in zip(bits, errs):
        assert e <= max(2.0 ** (6 - b), 1e-14), (b, e)
    for (b0, e0), (b1, e1) in zip(zip(bits, errs), zip(bits[1:], errs[1:])):
        assert b1 >= b0 + 3 or b1 == 48
        assert e1 <= max(e0 * 0.25, 1e-13)


def test_crt_residues_exact_at_48_bits():
    """Inputs m 2^-40 with |m| < 2^47: with 14 moduli and a short contraction
    every input becomes an integer of up to 48 bits exactly, so the residue
    products and the Chinese-remainder rebuild are exact and only the final
    conversion to FP64 rounds (about one ulp of the result).  A residue pass
    whose quotient y / p were misrounded at that size would fail this."""
    labA, labB, labC = "ik", "kj", "ij"
    ext = {"i": 70, "k": 100, "j": 45}
    g = np.random.default_rng(29)
    lim = 2 ** 47 - 1
    A = np.asfortranarray(g.integers(-lim, lim, size=(70, 100)).astype(np.float64) * 2.0 ** -40)
    B = np.asfortranarray(g.integers(-lim, lim, size=(100, 45)).astype(np.float64) * 2.0 ** -40)
    got, info = _run(labA, labB, labC, A, B, "crt_int8", slices=14)
    assert info["split_bits"] == 48
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print("crt 48-bit inputs: componentwise error %.3e" % err)
    assert err <= 1e-15


def test_crt_long_contraction_reduces_partial_sums():
    """More than 2^16 contracted indices: the residue sums are reduced modulo
    p on the way (exact on integers, within the bound on real inputs)."""
    labA, labB, labC = "ik", "k", "i"
    ext = {"i": 131, "k": 70001}
    A, B = synth.make_operands(27, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "crt_int8")
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    A, B = synth.make_operands(28, labA, labB, ext, kind="uniform")
    got, info = _run(labA, labB, labC, A, B, "crt_int8")
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print("crt K=70001 %d bits: componentwise error %.3e" % (info["split_bits"], err))
    assert err <= SPLIT_TOL


def test_split_error_falls_with_digits():
    name, labA, labB, labC, ext = CASES[1]
    A, B = synth.make_operands(23, labA, labB, ext, kind="scaled_normal")
    ref, absr = reference(A, labA, B, labB, labC)
    for precision, digits, gain in (("split_bf16", range(1, 8), 2.0 ** -6), ("split_fp8", range(1, 9), 2.0 ** -3)):
        errs = []
        for S in digits:
            got, info = _run(labA, labB, labC, A, B, precision, slices=S)
            errs.append(componentwise_error(got, ref, absr))
        print(precision, ["%.2e" % e for e in errs])
        # each extra digit adds b+1 bits (9 for BF16, 5 for FP8) until FP64 rounding dominates
        for e0, e1 in zip(errs, errs[1:]):
            assert e1 <= max(e0 * gain, 1e-13)


def test_split_alpha_beta():
    name, labA, labB, labC, ext = CASES[0]
    A, B = synth.make_operands(24, labA, labB, ext, kind="integers")
    C0 = synth.integers([ext[l] for l in labC], 5)
    for precision in ("split_bf16", "split_fp8", "crt_int8"):
        got, _ = _run(labA, labB, labC, A, B, precision, alpha=-2.0, beta=0.5, C0=C0)
        assert np.array_equal(got, -2.0 * oracle.contract(A, labA, B, labB, labC) + 0.5 * C0)


def test_split_rejects_batch_and_too_many_digits():
    A = torch.zeros(3, 4, 5, dtype=torch.float64, device="cuda")
    B = torch.zeros(4, 6, 5, dtype=torch.float64, device="cuda")
    C = torch.zeros(3, 6, 5, dtype=torch.float64, device="cuda")
    with pytest.raises(tc.TCError) as e:
        tc.Plan.for_tensors(A, "ikx", B, "kjx", C, "ijx", precision="split_bf16")
    assert e.value.status == tc.TC_ERR_UNSUPPORTED
    with pytest.raises(tc.TCError) as e:
        tc.Plan.for_tensors(A[:, :, 0], "ik", B[:, :, 0], "kj", C[:, :, 0], "ij", precision="split_bf16",
                            split_slices=9)
    assert e.value.status == tc.TC_ERR_INVALID_ARG


# FP8 digits at the default S = 8 keep 4 + 5*7 = 39 bits of each input below its
# row's power-of-two scale.  Bounds held here (componentwise, against the
# compensated oracle): 1e-10 on uniform inputs, 1e-9 on inputs whose slices
# are scaled by 10^U(-3,3) (a row then mixes entries six decades apart, and
# the small ones keep fewer bits of their own).
FP8_TOL_UNIFORM = 1e-10
FP8_TOL_SCALED = 1e-9


@pytest.mark.parametrize("kind,tol", [("uniform", FP8_TOL_UNIFORM), ("scaled_normal", FP8_TOL_SCALED)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_fp8_default_meets_its_bound(case, kind, tol):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(32, labA, labB, ext, kind=kind)
    got, info = _run(labA, labB, labC, A, B, "split_fp8")
    assert info["split_slices"] == 8
    ref, absr = reference(A, labA, B, labB, labC)
    err = componentwise_error(got, ref, absr)
    print(name, kind, "fp8 S=8 componentwise error %.3e" % err)
    assert err <= tol


@pytest.mark.parametrize("precision", ["split_fp8", "split_bf16"])
def test_split_long_contraction_flushes_level_sums(precision):
    """A contracted range of 9000 indices: the FP8 kernel moves its FP32 level
    sums to FP64 every 4096 indices (BF16: every 64 to 256), so the flush runs
    twice and ends on a partial chunk.  Exact on integers (the FP32 level
    sums of up to 4096 products of digits below 2^4 stay below 2^24), within
    the bound otherwise."""
    labA, labB, labC = "ik", "kj", "ij"
    ext = {"i": 70, "k": 9000, "j": 50}
    A, B = synth.make_operands(33, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, precision)
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    # integers up to 2^4 in both inputs: the largest level-0 products of FP8
    # digits, summed over the whole flush chunk
    A = np.full((70, 9000), 15.0, order="F")
    B = np.full((9000, 50), -15.0, order="F")
    got, info = _run(labA, labB, labC, A, B, precision)
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
    tol = {"split_fp8": (FP8_TOL_UNIFORM, FP8_TOL_SCALED), "split_bf16": (SPLIT_TOL, SPLIT_TOL)}[precision]
    for kind, t in zip(("uniform", "scaled_normal"), tol):
        A, B = synth.make_operands(34, labA, labB, ext, kind=kind)
        got, info = _run(labA, labB, labC, A, B, precision)
        ref, absr = reference(A, labA, B, labB, labC)
        err = componentwise_error(got, ref, absr)
        print(precision, kind, "K=9000 componentwise error %.3e" % err)
        assert err <= t


@pytest.mark.timeout(300)
@pytest.mark.parametrize("K", [1_600_000, 1_700_000])
def test_split_bf16_very_long_contracted_range(K):
    """Five BF16 digits over 1.6 and 1.7 million contracted indices: the
    copy-fed digit GEMM addresses a tile's 128 rows of digits by 32-bit byte
    offsets, up to 2.03e9 bytes at K = 1.6e6; at K = 1.7e6 the rows would
    pass 2^31 bytes and the launch takes the register-staged kernel instead.
    Exact on integers."""
    labA, labB, labC = "ik", "kj", "ij"
    ext = {"i": 3, "k": K, "j": 2}
    A, B = synth.make_operands(35, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B, "split_bf16")
    assert info["split_slices"] == 5
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))
