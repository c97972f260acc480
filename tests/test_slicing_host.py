"""Host checks of the forced-slicing executor's argument handling (no GPU
call is reached: every case is rejected, or only counted, before a plan)."""
import pytest
import torch

from paper_1307_2100_amd import slicing


def test_rejects_bad_slicings_and_counts_calls():
    A = torch.zeros(3, 4, dtype=torch.float64)
    B = torch.zeros(4, 5, dtype=torch.float64)
    C = torch.zeros(3, 5, dtype=torch.float64)
    with pytest.raises(ValueError):
        slicing.run_sliced(A, "ak", B, "kb", C, "ab", "z")       # in neither input
    with pytest.raises(ValueError):
        slicing.run_sliced(A, "ak", B, "kb", C, "ab", "kk")      # sliced twice
    Z = torch.zeros(3, 0, dtype=torch.float64)
    with pytest.raises(ValueError):
        slicing.run_sliced(Z, "ak", torch.zeros(0, 5, dtype=torch.float64), "kb", C, "ab", "k")  # extent 0
    assert slicing.slice_count(A, "ak", B, "kb", "ab") == 15
    assert slicing.slice_count(A, "ak", B, "kb", "") == 1
    assert slicing.slice_count(A, "ak", B, "kb", "k") == 4
