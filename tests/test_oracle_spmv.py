"""The plain OpenMP CSR product of the CPU baseline against SciPy's product
and against a dense product of a tiny matrix written out by hand."""
import numpy as np
import scipy.sparse as sp

from oracle import cspmv


def test_hand_matrix():
    A = sp.csr_matrix(np.array([[2.0, 0.0, -1.0], [0.0, 0.0, 0.0], [0.5, 3.0, 0.0]]))
    y, used = cspmv.spmv(A, np.array([1.0, 2.0, 4.0]))
    np.testing.assert_array_equal(y, [2.0 - 4.0, 0.0, 0.5 + 6.0])
    assert used >= 1


def test_matches_scipy_random():
    A = sp.random(3000, 2500, density=0.005, format="csr", random_state=3)
    x = np.random.default_rng(1).normal(size=2500)
    y, _ = cspmv.spmv(A, x)
    np.testing.assert_allclose(y, A @ x, rtol=1e-13, atol=1e-13)
