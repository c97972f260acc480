"""The committed picker model (CPU only): the file is well formed, matches
the library's candidate table and feature count, and its FP64 forward pass
(oracle.mlp_ref) ranks candidates sensibly on shapes whose best recipe is not
in doubt."""
import os

import numpy as np
import pytest

from oracle import mlp_ref

tc = pytest.importorskip("paper_1307_2100_amd")
from paper_1307_2100_amd import picker  # noqa: E402

pytestmark = pytest.mark.skipif(not os.path.exists(picker.DEFAULT_MODEL), reason="no trained model in the package")


def _colmajor(labels, ext):
    shape = [ext[l] for l in labels]
    st, acc = [], 1
    for e in shape:
        st.append(acc)
        acc *= e
    return tc.Desc(shape, st, labels)


def _predict(params, mean, std, labA, labB, labC, ext):
    f, rule = tc.tc_picker_features(_colmajor(labA, ext), _colmajor(labB, ext), _colmajor(labC, ext))
    x = (np.array(f, dtype=np.float64) - mean) / std
    y, _ = mlp_ref.forward(params.astype(np.float64), x[None, :], tc.PICKER_FEATURES, picker.HIDDEN,
                           tc.PICKER_CANDIDATES)
    return y[0], rule


def test_model_file_matches_the_library():
    params, mean, std, doc = picker.load_model()
    assert params.size == mlp_ref.num_params(tc.PICKER_FEATURES, picker.HIDDEN, tc.PICKER_CANDIDATES)
    assert doc["train_shapes"] >= 50000 and doc["test_shapes"] >= 5000
    held = doc["eval_heldout"]
    # the recorded evaluation: the network beats the rules on held-out shapes
    assert held["gain_geomean_rules_over_pick"] > 1.0
    assert held["geomean_pick_over_best"] < held["geomean_rules_over_best"]


def test_model_prefers_matrix_cores_for_a_large_gemm_and_not_for_a_dot():
    params, mean, std, _ = picker.load_model()
    gemm = [c for c in range(tc.PICKER_CANDIDATES) if tc.tc_picker_candidate(c)[0] in (tc.TC_RECIPE_GEMM,
                                                                                     tc.TC_RECIPE_COPY_GEMM)]
    # a large class-1 GEMM-shaped contraction: a GEMM candidate (or the rules' own GEMM plan) must win
    y, _ = _predict(params, mean, std, "ik", "kj", "ij", {"i": 2048, "k": 2048, "j": 2048})
    best = int(np.argmin(y))
    assert best in gemm or best == tc.PICKER_CANDIDATES - 1, best
    # a long inner product: a memory-bound candidate or the rules must beat every GEMM tile
    y, _ = _predict(params, mean, std, "k", "k", "", {"k": 1 << 22})
    assert min(y[c] for c in range(tc.PICKER_CANDIDATES) if c not in gemm) < min(y[c] for c in gemm)


def test_corrupt_model_is_rejected(tmp_path):
    bad = tmp_path / "m.json"
    bad.write_text('{"format": "tc-picker-mlp", "n_in": 32, "hidden": 64, "n_out": 15, "candidates": []}')
    with pytest.raises(ValueError):
        picker.load_model(str(bad))
