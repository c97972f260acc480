"""The full batch workload in one persistent launch, checked against the
oracle: the two general-relativity grid contractions of the paper's Sec. 4.2
example (every tensor extent 4) on a 128^3 grid, plus 2000 random
contractions of rank 3-6 with extents uniform in [4, 64], random storage
orders and random contracted sets -- the shapes and launch configuration the
benchmark times (graph replay, autotuned tile configuration).

Inputs are integers in [-4, 4], so every sum is exact and each checked entry
must equal the oracle bit for bit.  Samples are stratified per contraction:
every entry of a contraction whose oracle costs little (|C| * K <= 2^21),
otherwise 24 random entries plus the first and last; 4096 random entries plus
the corners of each grid contraction."""
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


def _contracted(la, lb, lc, ext):
    return int(np.prod([ext[l] for l in la if l in lb and l not in lc])) if la else 1


def _samples(la, lb, lc, ext, g, n):
    shape = [ext[l] for l in lc]
    if not shape:
        return np.zeros((1, 0), dtype=np.int64)
    idx = np.stack([g.integers(0, e, n) for e in shape], axis=1)
    ends = np.array([[0] * len(shape), [e - 1 for e in shape]])
    return np.concatenate([idx, ends]).astype(np.int64)


def _check(entries, g):
    bad = []
    for i, e in enumerate(entries):
        la, lb, lc, ext = e["spec"]
        got = e["C"].cpu().numpy()
        size = int(np.prod([ext[l] for l in lc])) if lc else 1
        if size * _contracted(la, lb, lc, ext) <= 1 << 21:
            ref = oracle.contract(e["A"], la, e["B"], lb, lc)
            if not np.array_equal(got, ref):
                bad.append(i)
            continue
        idx = _samples(la, lb, lc, ext, g, 4096 if i < 2 else 24)
        s, _ = oracle.contract_entries(e["A"], la, e["B"], lb, lc, idx, with_abs=False)
        if not np.array_equal(got[tuple(idx.T)], s):
            bad.append(i)
    return bad


@pytest.mark.timeout(900)
def test_full_batch_workload_exact():
    g = np.random.default_rng(1307)
    specs = [synth.workload_gr_r(), synth.workload_gr_s()]
    specs += [synth.random_contraction(g, rank_range=(3, 6), ext_range=(4, 64), max_elems=1 << 20)
              for _ in range(2000)]
    entries = []
    for i, (la, lb, lc, ext) in enumerate(specs):
        A, B = synth.make_operands(500 + i, la, lb, ext, kind="integers")
        C = colmajor_zeros([ext[l] for l in lc])
        dA, dB = to_dev(A), to_dev(B)
        plan = tc.Plan.for_tensors(dA, la, dB, lb, C, lc)
        entries.append(dict(spec=(la, lb, lc, ext), A=A, B=B, dA=dA, dB=dB, C=C, plan=plan))
    print("2002 plans built; grid contractions on kernels %s" % [tc.KERNEL_NAMES[e["plan"].info.kernel]
                                                                  for e in entries[:2]], flush=True)
    batch = tc.Batch([e["plan"] for e in entries])
    for e in entries:
        e["plan"].close()
    As, Bs, Cs = [e["dA"] for e in entries], [e["dB"] for e in entries], [e["C"] for e in entries]
    # default tile configuration, graph replay
    batch.execute(As, Bs, Cs)
    torch.cuda.synchronize()
    print("batch of %d tasks executed" % batch.query()["ntasks"], flush=True)
    assert _check(entries, np.random.default_rng(5)) == []
    # the benchmark's configuration: autotuned tiles, pointers bound once, replayed twice
    best, ms = batch.autotune(As, Bs, Cs)
    batch.set_options(best, 1)
    batch.bind(As, Bs, Cs)
    for C in Cs:
        C.fill_(7.0)
    batch.run()
    batch.run()
    torch.cuda.synchronize()
    print("autotuned configuration %d: %.3f ms" % (best, ms), flush=True)
    assert _check(entries, np.random.default_rng(6)) == []
    batch.close()
