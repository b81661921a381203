"""CPU check of the differentiable solve's argument handling: a matrix with
stored zeros is refused before any device work (the library drops stored
zeros at setup, so their values could not change in later calls)."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")


def test_stored_zeros_are_refused():
    from paper_2009_06954_amd.autograd import LinearSolve
    A = sp.csr_matrix(np.array([[2.0, 1.0], [0.5, 3.0]]))
    A.data[1] = 0.0  # a stored zero
    assert A.nnz == 4
    with pytest.raises(ValueError, match="stored zeros"):
        LinearSolve(A)
