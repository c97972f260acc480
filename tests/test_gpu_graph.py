"""tc_execute captured in a HIP graph: every replay, with other eager work
and synchronisations in between, gives the eager result bit for bit, for
each kernel family (direct GEMM, COPY+GEMM, split-K GEMM with its
reduction, segmented DOT, the slab engine)."""
import numpy as np
import pytest

import synth

from gpu_util import colmajor_zeros, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

CASES = [
    ("gemm", "ikm", "kj", "ijm", {"i": 70, "k": 37, "m": 5, "j": 45}, "auto"),
    ("copy_gemm", "abg", "gah", "bh", {"a": 33, "b": 70, "g": 17, "h": 129}, "auto"),
    ("split_k", "ak", "kb", "ab", {"a": 383, "k": 2100, "b": 390}, "auto"),
    ("dot_segments", "abg", "abg", "", {"a": 40, "b": 170, "g": 9}, "auto"),
    ("slab", "acbdx", "cdx", "abx", {"a": 4, "b": 4, "c": 4, "d": 4, "x": 3000}, "auto"),
]


@pytest.mark.parametrize("name,la,lb,lc,ext,recipe", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_match_eager(name, la, lb, lc, ext, recipe):
    A, B = synth.make_operands(71, la, lb, ext, kind="uniform")
    dA, dB = to_dev(A), to_dev(B)
    C = colmajor_zeros([ext[l] for l in lc])
    plan = tc.Plan.for_tensors(dA, la, dB, lb, C, lc, recipe=recipe)
    try:
        ws = plan.workspace(C.device)
        stream = torch.cuda.current_stream()
        plan.execute(dA, dB, C, stream=stream, workspace=ws)
        torch.cuda.synchronize()
        eager = C.clone()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                plan.execute(dA, dB, C, stream=side, workspace=ws)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        other = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
        for k in range(3):
            C.fill_(float("nan"))
            other.mul_(1.0001)            # unrelated eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(C, eager), (name, k)
        del g
    finally:
        torch.cuda.synchronize()
        plan.close()
    print(name, plan.info.as_dict()["kernel_name"], "k_split", plan.info.k_split)
