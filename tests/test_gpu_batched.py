"""Batch-dominated contractions (many tiny contractions sharing a layout, as
in the general-relativity lattice example) through the slab kernel, in both
array-of-structures and structure-of-arrays storage, against the oracle."""
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

GRID = (10, 9, 7)


def _soa(labels):
    """Move the grid labels x, y, z to the front (batch index fastest)."""
    return "".join(l for l in labels if l in "xyz") + "".join(l for l in labels if l not in "xyz")


def _cases():
    out = []
    for name, w in (("gr_r", synth.workload_gr_r(GRID)), ("gr_s", synth.workload_gr_s(GRID))):
        labA, labB, labC, ext = w
        out.append((name + "_aos", labA, labB, labC, ext))
        out.append((name + "_soa", _soa(labA), _soa(labB), _soa(labC), ext))
    out.append(("mixed", _soa("acbdxyz"), "cdxyz", "abxyz", synth.workload_gr_r(GRID)[3]))
    out.append(("batch_mid", "axbc", "cxd", "adxb", {"a": 3, "b": 5, "c": 6, "d": 7, "x": 500}))
    return out


CASES = _cases()


def _run(labA, labB, labC, A, B, alpha=1.0, beta=0.0, C0=None):
    dA, dB = to_dev(A), to_dev(B)
    shape = [dict(zip(labA, A.shape), **dict(zip(labB, B.shape)))[l] for l in labC]
    C = colmajor_zeros(shape)
    if C0 is not None:
        C.copy_(to_dev(C0))
    plan = tc.Plan.for_tensors(dA, labA, dB, labB, C, labC)
    plan.execute(dA, dB, C, alpha, beta)
    torch.cuda.synchronize()
    info = plan.info.as_dict()
    plan.close()
    return C.cpu().numpy(), info


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_batched_exact_on_integers(case):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(31, labA, labB, ext, kind="integers")
    got, info = _run(labA, labB, labC, A, B)
    assert info["kernel_name"] == "batched_small", info
    assert np.array_equal(got, oracle.contract(A, labA, B, labB, labC))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_batched_uniform_alpha_beta(case):
    name, labA, labB, labC, ext = case
    A, B = synth.make_operands(32, labA, labB, ext, kind="uniform")
    C0 = synth.uniform([ext[l] for l in labC], 33)
    got, info = _run(labA, labB, labC, A, B, alpha=1.5, beta=-0.5, C0=C0)
    ref, absr = reference(A, labA, B, labB, labC, alpha=1.5, beta=-0.5, C0=C0)
    assert componentwise_error(got, ref, absr) <= FP64_TOL
