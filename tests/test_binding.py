"""CPU checks of the Python binding's argument validation: tensors that would
make the library read or write device memory out of range (wrong device, dtype,
layout, length or column count) are rejected before any library call."""
import numpy as np
import pytest
import torch

import paper_2609_31477_amd as mf


def test_check_vectors_accepts_and_counts():
    assert mf.check_vectors(torch.zeros(5, dtype=torch.float64), 5, "b", require_cuda=False) == 1
    assert mf.check_vectors(torch.zeros(3, 5, dtype=torch.float64), 5, "b", require_cuda=False) == 3


@pytest.mark.parametrize("bad,exc", [
    (torch.zeros(5, dtype=torch.float32), TypeError),           # wrong dtype
    (torch.zeros(5, 2, dtype=torch.float64).t(), TypeError),    # not contiguous
    (torch.zeros(4, dtype=torch.float64), ValueError),          # short
    (torch.zeros(2, 2, 5, dtype=torch.float64), ValueError),    # too many dimensions
    (np.zeros(5), TypeError),                                    # not a tensor
])
def test_check_vectors_rejects(bad, exc):
    with pytest.raises(exc):
        mf.check_vectors(bad, 5, "b", require_cuda=False)


def test_check_vectors_column_count_and_device():
    with pytest.raises(ValueError):
        mf.check_vectors(torch.zeros(2, 5, dtype=torch.float64), 5, "x", nrhs=3, require_cuda=False)
    with pytest.raises(TypeError):
        mf.check_vectors(torch.zeros(5, dtype=torch.float64), 5, "b")  # a CPU tensor


class _Dummy:
    """Stands for a factored handle: any library call on it would fail loudly."""
    n = 5
    options = None


def test_numeric_solve_rejects_cpu_and_bad_x_before_the_library():
    num = mf.Numeric(_Dummy())
    with pytest.raises(TypeError):
        num.solve(torch.zeros(5, dtype=torch.float64))


def test_batch_solve_rejects_before_the_library():
    B = mf.Batch.__new__(mf.Batch)  # no library handle: validation must come first
    B.syms = [_Dummy(), _Dummy()]
    B.ns = [5, 5]
    B._num = None
    with pytest.raises(ValueError):
        B.solve([torch.zeros(5, dtype=torch.float64)])                  # one tensor for two systems
    with pytest.raises(TypeError):
        B.solve([torch.zeros(5, dtype=torch.float64)] * 2)              # CPU tensors
