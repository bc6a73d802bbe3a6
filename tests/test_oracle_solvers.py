"""Pins of the oracle's reference solves."""
import numpy as np

import workloads as W
from oracle import solvers as S
from oracle.mesh import MacroMesh

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)


def test_manufactured_solution_recovered():
    mesh = MacroMesh(W.kuhn6(), 2)
    k = W.exp_fourier_coefficient(mesh.xyz, W.rng_for(2, 0), 16, 1.0)
    A, dof = S.reduced_system(mesh, k, EFORM)
    rng = np.random.default_rng(3)
    xs = rng.uniform(-1, 1, A.shape[0])
    x = S.direct_solve(A, A @ xs)
    np.testing.assert_allclose(x, xs, rtol=1e-10, atol=1e-10)
    xc, it = S.block_jacobi_cg(A, A @ xs, rtol=1e-12)
    np.testing.assert_allclose(xc, xs, rtol=1e-8, atol=1e-8)
    assert 0 < it < A.shape[0]


def test_block_jacobi_is_spd_and_blockwise():
    mesh = MacroMesh(W.unit_tet(), 3)
    k = W.sine_coefficient(mesh.xyz)
    A, _ = S.reduced_system(mesh, k, dict(mu0=1.0, lam1=1.0))
    M = S.block_jacobi_inverse(A).toarray()
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    D = A.toarray()
    for i in range(0, A.shape[0], 3):
        np.testing.assert_allclose(M[i:i + 3, i:i + 3] @ D[i:i + 3, i:i + 3], np.eye(3), atol=1e-10)
