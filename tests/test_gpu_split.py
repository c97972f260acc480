"""Split-precision contractions (FP64 digits on BF16 / FP8 matrix cores)
against the compensated FP64 oracle.

Integer-valued inputs in [-4, 4] fit in one digit, so every product and sum
is exact and the result must equal the oracle bit for bit.  Otherwise the
componentwise error must stay within the bound of the digit count: BF16 with
the default 5 digits (8 + 4x9 = 44 bits per input) is held to 1e-10, also on
inputs whose slices are scaled by 10^U(-3,3)."""
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


def _run(labA, labB, labC, A, B, precision, slices=0, alpha=1.0, beta=0.0, C0=None):
    dA, dB = to_dev(A), to_dev(B)
    shape = [dict(zip(labA, A.shape), **dict(zip(labB, B.shape)))[l] for l in labC]
    C = colmajor_zeros(shape)
    if C0 is not None:
        C.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, precision=precision, split_slices=slices)
    plan.execute(dA, dB, C, alpha, beta)
    torch.cuda.synchronize()
    info = plan.info.as_dict()
    plan.close()
    return C.cpu().numpy(), info


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp8"])
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
    for precision in ("split_bf16", "split_fp8"):
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
