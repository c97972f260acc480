"""Full-size coupled-cluster contractions on the GPU, in the launch
configuration the benchmark times, checked against the compensated oracle on
sampled outputs: one output inside every 64 x 64 block of the kernel's
(M, N) output grid -- so every GEMM tile of every configuration used here
(FP64 256 x 128, BF16 128 x 64, INT8 residues 256 x 256) holds at least one
-- plus the corners of C.

* v = 128, o = 32, uniform [-1, 1] inputs: FP64.
* v = 192, o = 48, N(0,1) inputs scaled per last-index slice by 10^U(-3,3)
  (the precision workload): FP64, split BF16 digits, split FP8 digits and
  INT8 residues, each held to its bound (FP64 1e-12, BF16 and residues
  1e-10, FP8 1e-9 on these scaled inputs)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import FP64_TOL, colmajor_zeros, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

# the kernel's row (M) and column (N) index groups, in fused order; C's
# stride-1 index a is free in A, so the kernels take B as their first input
GROUPS = {"cc_a": ("ij", "ab"), "cc_b": ("bj", "ai")}
TOL = {"f64": FP64_TOL, "split_bf16": 1e-10, "crt_int8": 1e-10, "split_fp8": 1e-9}


def block_samples(ext, labC, mlabs, nlabs, block, seed):
    """One random output in every block x block square of the (M, N) grid,
    M and N decoded column-major over mlabs / nlabs, plus C's corners."""
    g = np.random.default_rng(seed)
    M = int(np.prod([ext[l] for l in mlabs]))
    N = int(np.prod([ext[l] for l in nlabs]))
    m0, n0 = np.meshgrid(np.arange(0, M, block), np.arange(0, N, block), indexing="ij")
    m = (m0 + (g.random(m0.shape) * np.minimum(block, M - m0)).astype(np.int64)).ravel()
    n = (n0 + (g.random(n0.shape) * np.minimum(block, N - n0)).astype(np.int64)).ravel()
    val = {}
    for labs, lin in ((mlabs, m), (nlabs, n)):
        for l in labs:
            val[l] = lin % ext[l]
            lin = lin // ext[l]
    idx = np.stack([val[l] for l in labC], axis=1)
    shape = [ext[l] for l in labC]
    corners = np.array([[(e - 1) * ((c >> d) & 1) for d, e in enumerate(shape)] for c in range(1 << len(shape))])
    return np.concatenate([idx, corners]).astype(np.int64)


def check(which, A, B, labA, labB, labC, ext, dA, dB, precision, idx, ref, tol):
    shape = [ext[l] for l in labC]
    C = colmajor_zeros(shape)
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC, precision=precision)
    info = plan.info
    print(which, precision, info.as_dict(), flush=True)
    assert info.swapped == 1
    assert (info.M, info.N) == tuple(int(np.prod([ext[l] for l in g])) for g in GROUPS[which])
    plan.execute(dA, dB, C)
    torch.cuda.synchronize()
    got = C.cpu().numpy()[tuple(idx.T)]
    plan.close()
    del C
    s, a = ref
    err = float(np.max(np.abs(got - s) / a))
    print(which, precision, "componentwise error %.3e on %d sampled outputs" % (err, len(idx)), flush=True)
    assert err <= tol
    return err


@pytest.mark.parametrize("which", ["cc_a", "cc_b"])
def test_coupled_cluster_v128_every_tile(which):
    labA, labB, labC, ext = synth.workload_cc_a() if which == "cc_a" else synth.workload_cc_b()
    A, B = synth.make_operands(1, labA, labB, ext, kind="uniform")
    idx = block_samples(ext, labC, *GROUPS[which], 64, 5)
    ref = oracle.contract_entries(A, labA, B, labB, labC, idx)
    check(which, A, B, labA, labB, labC, ext, to_dev(A), to_dev(B), "f64", idx, ref, FP64_TOL)


_C2 = {}


def c2_inputs(which):
    """Inputs of the precision workload, on the host and the device, and the
    oracle's sums on the sampled outputs (computed once per contraction)."""
    if which not in _C2:
        _C2.clear()
        torch.cuda.empty_cache()
        spec = synth.workload_cc_a(192, 48) if which == "cc_a" else synth.workload_cc_b(192, 48)
        labA, labB, labC, ext = spec
        A, B = synth.make_operands(21 if which == "cc_a" else 22, labA, labB, ext, kind="scaled_normal")
        idx = block_samples(ext, labC, *GROUPS[which], 64, 7)
        ref = oracle.contract_entries(A, labA, B, labB, labC, idx)
        _C2[which] = (spec, A, B, to_dev(A), to_dev(B), idx, ref)
    return _C2[which]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["f64", "split_bf16", "split_fp8", "crt_int8"])
@pytest.mark.parametrize("which", ["cc_a", "cc_b"])
def test_precision_workload_v192_every_tile(which, precision):
    (labA, labB, labC, ext), A, B, dA, dB, idx, ref = c2_inputs(which)
    check(which, A, B, labA, labB, labC, ext, dA, dB, precision, idx, ref, TOL[precision])
    if which == "cc_b" and precision == "crt_int8":
        _C2.clear()
        torch.cuda.empty_cache()
