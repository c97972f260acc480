"""tc_execute_noalloc (the entry point that takes its workspace from the
library's fixed device array) against tc_execute with an allocated
workspace, through the C ABI: same plans, same inputs, bit-identical outputs,
on two calls in a row whose second has the smaller input (so it runs over the
first call's leftovers in the array), and integer inputs so both also equal
the oracle exactly."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import colmajor_zeros, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

# (name, labA, labB, labC, larger extents, smaller extents, plan options);
# every plan here needs a workspace: the copy of COPY+GEMM, split-K partial
# tiles, segment partials of the lanes kernels, or split-precision planes
CASES = [
    ("copy_gemm", "abg", "gah", "bh", {"a": 90, "b": 70, "g": 41, "h": 129}, {"a": 33, "b": 20, "g": 17, "h": 31},
     dict(recipe="copy_gemm")),
    ("split_k", "ak", "kb", "ab", {"a": 30, "k": 2100, "b": 600}, {"a": 20, "k": 3000, "b": 100}, dict()),
    ("lanes_segments", "abg", "bg", "a", {"a": 40, "b": 300, "g": 200}, {"a": 9, "b": 70, "g": 130}, dict()),
    ("split_bf16", "abcd", "cdij", "abij", {"a": 20, "b": 19, "c": 18, "d": 17, "i": 6, "j": 7},
     {"a": 9, "b": 5, "c": 7, "d": 3, "i": 4, "j": 3}, dict(precision="split_bf16")),
    ("crt_int8", "akic", "kbcj", "abij", {"a": 21, "k": 5, "i": 6, "c": 19, "b": 17, "j": 4},
     {"a": 5, "k": 3, "i": 2, "c": 7, "b": 6, "j": 3}, dict(precision="crt_int8")),
]


def _one(labA, labB, labC, ext, opts, seed, beta):
    A, B = synth.make_operands(seed, labA, labB, ext, kind="integers")
    shape = [ext[l] for l in labC]
    C0 = synth.integers(shape, synth.seed_for(seed, 2)) if beta else None
    dA, dB = to_dev(A), to_dev(B)
    C_ref = colmajor_zeros(shape)
    C_na = colmajor_zeros(shape)
    if C0 is not None:
        C_ref.copy_(to_dev(C0))
        C_na.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C_ref, labC, **opts)
    info = plan.info
    assert 0 < info.workspace_bytes <= tc.NOALLOC_SCRATCH_BYTES, info.as_dict()
    print("noalloc", labA, labB, labC, ext, opts, "workspace", info.workspace_bytes, flush=True)
    plan.execute(dA, dB, C_ref, 1.0, beta)
    plan.execute_noalloc(dA, dB, C_na, 1.0, beta)
    torch.cuda.synchronize()
    got, ref = C_na.cpu().numpy(), C_ref.cpu().numpy()
    plan.close()
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    want = oracle.contract(A, labA, B, labB, labC)
    if C0 is not None:
        want = want + beta * C0
    assert np.array_equal(got, want.reshape(got.shape))
    return info


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_execute_twice(case):
    name, labA, labB, labC, big, small, opts = case
    info_big = _one(labA, labB, labC, big, opts, 31, 0.0)
    info_small = _one(labA, labB, labC, small, opts, 32, 2.0)
    assert info_small.workspace_bytes < info_big.workspace_bytes
    if name == "split_k":
        assert info_big.k_split > 1 and info_small.k_split > 1
    if name == "copy_gemm":
        assert info_big.copy_operand >= 0


def test_noalloc_without_workspace():
    """A plan that needs no workspace runs through the entry point too."""
    labA, labB, labC = "ik", "kj", "ij"
    ext = {"i": 70, "k": 33, "j": 45}
    A, B = synth.make_operands(33, labA, labB, ext, kind="integers")
    dA, dB = to_dev(A), to_dev(B)
    C = colmajor_zeros([70, 45])
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC)
    assert plan.info.workspace_bytes == 0
    plan.execute_noalloc(dA, dB, C)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), oracle.contract(A, labA, B, labB, labC))
    plan.close()


def test_noalloc_rejects_plan_beyond_the_array():
    """A plan whose workspace exceeds the array is refused before anything is
    enqueued (C keeps its contents)."""
    labA, labB, labC = "abg", "gah", "bh"
    ext = {"a": 300, "b": 4, "g": 8000, "h": 5}  # the copied operand, A, holds 9.6 M doubles (77 MB)
    A, B = synth.make_operands(34, labA, labB, ext, kind="integers")
    dA, dB = to_dev(A), to_dev(B)
    C = colmajor_zeros([4, 5])
    C.fill_(7.0)
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, recipe="copy_gemm")
    if plan.info.workspace_bytes <= tc.NOALLOC_SCRATCH_BYTES:
        plan.close()
        pytest.skip("copy workspace %d bytes fits the array" % plan.info.workspace_bytes)
    with pytest.raises(tc.TCError) as exc:
        plan.execute_noalloc(dA, dB, C)
    assert exc.value.status == tc.TC_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert float(C.min()) == 7.0 and float(C.max()) == 7.0
    plan.close()
