"""GPU parity of the forced-slicing executor (the paper's slice loops of
Sec. 2.4, one library call per slice) against the CPU oracle: bit-exact on
integer inputs for GEMM, GEMV, GER and DOT slicings, sliced free, contracted
and batch indices, and beta != 0 (the first contracted slice takes beta, the
rest accumulate)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import colmajor_zeros, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1307_2100_amd import slicing  # noqa: E402

CASES = [
    ("abg", "hbg", "ah", {"a": 9, "b": 7, "g": 5, "h": 6}, ["", "g", "b", "hg", "bg", "ah", "a", "gbh"]),
    ("abg", "gah", "bh", {"a": 9, "b": 7, "g": 5, "h": 6}, ["g", "a", "ag", "bh"]),
    ("acbdx", "cdx", "abx", {"a": 4, "b": 3, "c": 5, "d": 2, "x": 7}, ["x", "xc", "dx"]),
    ("iajb", "jgid", "abgd", {"i": 5, "j": 4, "a": 3, "b": 2, "g": 6, "d": 3}, ["ij", "ab", "i"]),
]


@pytest.mark.parametrize("la,lb,lc,ext,sl", [(c[0], c[1], c[2], c[3], s) for c in CASES for s in c[4]])
def test_sliced_matches_oracle(la, lb, lc, ext, sl):
    A, B = synth.make_operands(21, la, lb, ext, kind="integers")
    C0 = synth.integers([ext[l] for l in lc], 22)
    C = colmajor_zeros([ext[l] for l in lc])
    C.copy_(to_dev(C0))
    calls = slicing.run_sliced(to_dev(A), la, to_dev(B), lb, C, lc, sl, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    assert calls == int(np.prod([ext[l] for l in sl]))
    want = 2.0 * oracle.contract(A, la, B, lb, lc) - C0
    assert np.array_equal(C.cpu().numpy(), want)

