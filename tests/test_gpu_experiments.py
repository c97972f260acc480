"""GPU checks of the experiment driver (Sec. 4 studies with forced recipes,
and the layout advice of Sec. 3.3) at small sizes: every forced recipe and
the suggested layout agree with the rules' result (the driver raises
otherwise), and each recipe runs what it was asked for."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1307_2100_amd import experiments  # noqa: E402


@pytest.mark.parametrize("study,la,lb,lc,ext", [
    ("square", "abg", "hbg", "ah", {l: 37 for l in "abgh"}),
    ("square", "abg", "gah", "bh", {l: 37 for l in "abgh"}),
    ("cc", "iaj", "icjd", "acd", {"i": 70, "j": 65, "a": 6, "c": 7, "d": 5}),
    ("gr", "iaj", "icjd", "acd", {"i": 4, "j": 4, "a": 40, "c": 33, "d": 21}),
])
def test_forced_recipes_agree(study, la, lb, lc, ext):
    rows = experiments.run_recipes(study, la, lb, lc, ext, experiments.RECIPES[study], seed=5)
    assert [r["recipe"] for r in rows] == ["auto"] + list(experiments.RECIPES[study])
    for r in rows[1:]:
        assert r["ran"] == r["recipe"] and r["max_diff_over_K"] <= 1e-12


def test_layout_advice_rows():
    rows = experiments.run_layout("cdab", "dcij", "abij", {"a": 20, "b": 9, "c": 12, "d": 7, "i": 5, "j": 6}, seed=6)
    given, suggested = rows
    assert given["paper_class"] == 31 and given["ran"] == "copy_gemm"
    assert suggested["paper_class"] == 32 and suggested["ran"] == "gemm" and suggested["copy_operand"] == -1
    assert suggested["max_diff_over_K"] <= 1e-12
