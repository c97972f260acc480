"""GPU parity of multi-operand chains (paper_1307_2100_amd.chain) against the
CPU oracle applied pairwise in operand order: bit-exact on integer inputs,
whatever order and intermediate layouts the chain takes."""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1307_2100_amd import chain  # noqa: E402

SPECS = [
    ("abcd,ae,bf->efcd", {"a": 6, "b": 5, "c": 4, "d": 3, "e": 7, "f": 2}),     # raising two indices
    ("ae,bf,abcd->efcd", {"a": 6, "b": 5, "c": 4, "d": 3, "e": 7, "f": 2}),
    ("ij,jk,kl,lm->im", {"i": 9, "j": 2, "k": 30, "l": 3, "m": 11}),
    ("aix,ibx,bcx,c->ax", {"a": 4, "i": 6, "b": 5, "c": 7, "x": 3}),           # a batch index throughout
    ("ab,bc,cd,de,ea->", {"a": 3, "b": 8, "c": 2, "d": 9, "e": 4}),           # a trace: scalar result
    ("pq,qrs,st,trp,u->u", {"p": 3, "q": 4, "r": 2, "s": 5, "t": 6, "u": 2}),
]


def oracle_chain(arrays, labels, out):
    """Pairwise in operand order, keeping every label still needed."""
    cur, lab = arrays[0], labels[0]
    for k in range(1, len(arrays)):
        later = set("".join(labels[k + 1:])) | set(out)
        keep = "".join(l for l in dict.fromkeys(lab + labels[k]) if l in later)
        if k == len(arrays) - 1:
            keep = out
        cur, lab = oracle.contract(cur, lab, arrays[k], labels[k], keep), keep
    return cur


@pytest.mark.parametrize("order", ["optimal", "left"])
@pytest.mark.parametrize("expr,ext", SPECS)
def test_chain_matches_oracle(expr, ext, order):
    ins, out = expr.split("->")
    labels = ins.split(",")
    arrays = [synth.integers([ext[l] for l in lab], 30 + i, lo=-2, hi=2) for i, lab in enumerate(labels)]
    got = chain.contract_chain([(to_dev(a), lab) for a, lab in zip(arrays, labels)], out, order=order)
    want = oracle_chain(arrays, labels, out)
    assert got.shape == tuple(ext[l] for l in out)
    assert np.array_equal(got.cpu().numpy(), want)


def test_chain_writes_into_out():
    ext = {"a": 6, "b": 5, "c": 4, "d": 3, "e": 7, "f": 2}
    labels = ["abcd", "ae", "bf"]
    arrays = [synth.integers([ext[l] for l in lab], 40 + i, lo=-2, hi=2) for i, lab in enumerate(labels)]
    out = torch.zeros([ext[l] for l in "efcd"], dtype=torch.float64, device="cuda")
    r = chain.contract_chain([(to_dev(a), lab) for a, lab in zip(arrays, labels)], "efcd", out=out)
    assert r is out
    assert np.array_equal(out.cpu().numpy(), oracle_chain(arrays, labels, "efcd"))


def test_planned_chain_runs_again_on_new_operands():
    ext = {"i": 9, "j": 2, "k": 30, "l": 3, "m": 11}
    labels = ["ij", "jk", "kl", "lm"]
    first = [synth.integers([ext[l] for l in lab], 50 + i, lo=-2, hi=2) for i, lab in enumerate(labels)]
    second = [synth.integers([ext[l] for l in lab], 60 + i, lo=-2, hi=2) for i, lab in enumerate(labels)]
    ch = chain.Chain([(to_dev(a), lab) for a, lab in zip(first, labels)], "im")
    try:
        for arrays in (first, second):
            got = ch.execute([to_dev(a) for a in arrays])
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), oracle_chain(arrays, labels, "im"))
    finally:
        ch.close()
