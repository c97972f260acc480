"""Full-size coupled-cluster contractions (v = 128, o = 32) on the GPU,
checked on sampled outputs against the compensated oracle, in the launch
configuration the benchmark times."""
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


def sample_indices(shape, n, seed):
    g = np.random.default_rng(seed)
    idx = np.stack([g.integers(0, e, n) for e in shape], axis=1)
    # plus the corners
    corners = np.array([[0] * len(shape), [e - 1 for e in shape]])
    return np.concatenate([idx, corners])


@pytest.mark.parametrize("which", ["cc_a", "cc_b"])
def test_coupled_cluster_full_size_sampled(which):
    labA, labB, labC, ext = synth.workload_cc_a() if which == "cc_a" else synth.workload_cc_b()
    A, B = synth.make_operands(1, labA, labB, ext, kind="uniform")
    dA, dB = to_dev(A), to_dev(B)
    shape = [ext[l] for l in labC]
    C = colmajor_zeros(shape)
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC)
    print(which, plan.info.as_dict())
    plan.execute(dA, dB, C)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    idx = sample_indices(shape, 2048, 5)
    s, a = oracle.contract_entries(A, labA, B, labB, labC, idx)
    g = got[tuple(idx.T)]
    err = float(np.max(np.abs(g - s) / a))
    print(which, "sampled componentwise error %.3e" % err)
    assert err <= FP64_TOL
    plan.close()
