"""Persistent batches: many contractions of any shapes (random ranks, extents,
storage orders and contracted sets, plus general-relativity-shaped grid
contractions) in one launch, graph-replayed, against the oracle."""
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


def _make_batch(count, seed, kind="integers"):
    g = np.random.default_rng(seed)
    specs = [synth.workload_gr_r((6, 5, 4)), synth.workload_gr_s((6, 5, 4)),
             ("akb", "kbc", "ac", {"a": 31, "k": 300, "b": 37, "c": 5}),      # split-K tasks
             ("ikm", "kj", "ijm", {"i": 70, "k": 3000, "m": 2, "j": 9}),
             # memory-bound shapes kept on their lanes kernels, long contracted ranges in segments
             ("ki", "k", "i", {"k": 40000, "i": 7}),                             # lanes over k, 3 segments
             ("kb", "kb", "b", {"k": 50000, "b": 3}),                            # inner products per b
             ("ik", "k", "i", {"i": 300, "k": 3000}),                            # lanes over outputs, segments
             ("ik", "kj", "ij", {"i": 600, "k": 300, "j": 1}),
             # inner products over two contracted modes whose stride-1 modes differ (block tables,
             # ragged blocks), and the same with a zero extent (an empty sum: plain tables)
             ("kmi", "mki", "i", {"k": 37, "m": 30, "i": 3}),
             ("kmi", "mki", "i", {"k": 0, "m": 30, "i": 3})]
    for _ in range(count):
        specs.append(synth.random_contraction(g, rank_range=(3, 6), ext_range=(2, 9), max_elems=20000,
                                              p_outer=0.03, allow_batch=True))
    entries = []
    for i, (la, lb, lc, ext) in enumerate(specs):
        A, B = synth.make_operands(200 + i, la, lb, ext, kind=kind)
        C = colmajor_zeros([ext[l] for l in lc])
        dA, dB = to_dev(A), to_dev(B)
        plan = tc.Plan.for_tensors(dA, la, dB, lb, C, lc)
        entries.append(dict(spec=(la, lb, lc), A=A, B=B, dA=dA, dB=dB, C=C, plan=plan))
    batch = tc.Batch([e["plan"] for e in entries])
    for e in entries:
        e["plan"].close()      # a batch keeps what it needs
    return batch, entries


def _check_exact(entries, alphas=None):
    for i, e in enumerate(entries):
        la, lb, lc = e["spec"]
        ref = oracle.contract(e["A"], la, e["B"], lb, lc)
        if alphas is not None:
            ref = alphas[i] * ref
        assert np.array_equal(e["C"].cpu().numpy(), ref), (i, e["spec"])


def test_memory_bound_shapes_keep_their_lanes_kernels():
    for la, lb, lc, ext, kernel in (("ki", "k", "i", {"k": 40000, "i": 7}, "lanes_over_k"),
                                    ("kb", "kb", "b", {"k": 50000, "b": 3}, "lanes_over_k"),
                                    ("ik", "k", "i", {"i": 300, "k": 3000}, "lanes_over_outputs")):
        shapes = [[ext[l] for l in x] for x in (la, lb, lc)]
        descs = []
        for x, lab in zip(shapes, (la, lb, lc)):
            st, acc = [], 1
            for e in x:
                st.append(acc)
                acc *= e
            descs.append(tc.Desc(x, st, lab))
        assert tc.KERNEL_NAMES[tc.tc_analyze(*descs).kernel] == kernel, (la, lb, lc)


def test_batch_matches_oracle_graph_and_eager():
    batch, entries = _make_batch(60, 7)
    print(batch.query())
    for use_graph in (1, 0):
        for e in entries:
            e["C"].zero_()
        batch.set_options(-1, use_graph)
        batch.execute([e["dA"] for e in entries], [e["dB"] for e in entries], [e["C"] for e in entries])
        torch.cuda.synchronize()
        _check_exact(entries)
    batch.close()


def test_graph_replays_agree_with_eager_runs():
    """Replay the captured graph several times with new input values and
    different scalars, with eager work and synchronisations in between; each
    replay must equal an eager run of the same inputs."""
    batch, entries = _make_batch(25, 11)
    As, Bs, Cs = [e["dA"] for e in entries], [e["dB"] for e in entries], [e["C"] for e in entries]
    for rep in range(4):
        for i, e in enumerate(entries):
            e["dA"].copy_(to_dev(synth.integers(e["A"].shape, 1000 * rep + i)))
            e["A"] = e["dA"].cpu().numpy()
        alphas = [float(rep + 1)] * len(entries)
        batch.set_options(-1, 0)
        batch.execute(As, Bs, Cs, alphas=alphas)
        torch.cuda.synchronize()
        eager = [c.clone() for c in Cs]
        junk = torch.randn(1000, device="cuda").sum()     # unrelated eager work
        for c in Cs:
            c.fill_(7.0)
        batch.set_options(-1, 1)
        batch.execute(As, Bs, Cs, alphas=alphas)
        torch.cuda.synchronize()
        del junk
        for c, r in zip(Cs, eager):
            assert torch.equal(c, r)
        _check_exact(entries, alphas)
    batch.close()


def test_autotune_keeps_results_and_new_buffers():
    batch, entries = _make_batch(30, 13)
    As, Bs, Cs = [e["dA"] for e in entries], [e["dB"] for e in entries], [e["C"] for e in entries]
    best, ms = batch.autotune(As, Bs, Cs)
    assert 0 <= best < 6 and ms > 0
    assert batch.query()["tile_config"] == best
    # fresh output buffers: the graph reads pointers at every replay
    Cs2 = [torch.zeros_like(c) for c in Cs]
    for e, c in zip(entries, Cs2):
        e["C"] = c
    batch.set_options(-1, 1)
    batch.execute(As, Bs, Cs2)
    torch.cuda.synchronize()
    _check_exact(entries)
    batch.close()
