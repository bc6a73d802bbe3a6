"""P1 local stiffness tensors of the vector-valued forms (paper Sec. 2).

For an element t with nodal basis functions phi_a and canonical unit vectors
e_l, the local stiffness tensor of a form D (D = eps or div) is

    (a^t_ij)_{lm} = int_t ( D(phi_j e_l), D(phi_i e_m) ) dx

(the tensor used in the proof of the Lemma and, summed over elements, in eq.
stiffcontribution).  i is the test node, j the trial node, l the trial and m
the test component.  Because P1 gradients are constant the integral is the
element volume times the pointwise product.

The operator of the paper's elasticity problem (eq. bilinearformstd) is
2 mu (eps(u), eps(v)) + lam (div u, div v); ``form_tensor`` returns that
combination for given (mu, lam).

Parity: pinned by tests (zero block-row sums, symmetry a_ij = a_ji^T, rigid
body modes in the kernel, the energy of an affine displacement field, the
reflection relation and the closed form of the antisymmetric part eq.
localcorr3d from Sec. 2.4).
"""
from __future__ import annotations

import numpy as np


def p1_gradients(X: np.ndarray):
    """Gradients of the barycentric basis on elements X (T,4,3).

    Returns (grad (T,4,3), vol (T,)).  With M the matrix whose columns are
    x_a - x_0 (a = 1..3), lambda = M^{-1}(x - x_0), so the rows of M^{-1} are
    the gradients of lambda_1..3 and grad lambda_0 = -(their sum).
    """
    X = np.asarray(X, dtype=np.float64)
    M = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    Minv = np.linalg.inv(M)
    g = np.empty(X.shape)
    g[:, 1:, :] = Minv
    g[:, 0, :] = -Minv.sum(axis=1)
    vol = np.abs(np.linalg.det(M)) / 6.0
    return g, vol


def sym_grad_basis(g: np.ndarray) -> np.ndarray:
    """eps(phi_a e_l) as explicit 3x3 matrices: shape (T, 4, 3, 3, 3) with
    indices [t, a, l, p, q] = 1/2 (delta_lp d_q phi_a + delta_lq d_p phi_a)."""
    T = g.shape[0]
    eye = np.eye(3)
    grad_u = np.einsum("lp,taq->talpq", eye, g)        # d_q (phi_a e_l)_p
    return 0.5 * (grad_u + np.transpose(grad_u, (0, 1, 2, 4, 3))).reshape(T, 4, 3, 3, 3)


def eps_tensor(g: np.ndarray, vol: np.ndarray) -> np.ndarray:
    """(a^t_ij)_{lm} for D = eps: [t, i, j, l, m]."""
    E = sym_grad_basis(g)
    return vol[:, None, None, None, None] * np.einsum("tjlpq,timpq->tijlm", E, E)


def div_tensor(g: np.ndarray, vol: np.ndarray) -> np.ndarray:
    """(a^t_ij)_{lm} for D = div: div(phi_j e_l) div(phi_i e_m) = g_jl g_im."""
    return vol[:, None, None, None, None] * np.einsum("tjl,tim->tijlm", g, g)


def form_tensor(X: np.ndarray, mu: float, lam: float) -> np.ndarray:
    """Local tensor of 2 mu (eps, eps) + lam (div, div) on elements X."""
    g, vol = p1_gradients(X)
    out = np.zeros((X.shape[0], 4, 4, 3, 3))
    if mu != 0.0:
        out += 2.0 * mu * eps_tensor(g, vol)
    if lam != 0.0:
        out += lam * div_tensor(g, vol)
    return out


def sym_part(a: np.ndarray) -> np.ndarray:
    """a^{s} = 1/2 (a + a^T) over the component indices (last two axes)."""
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def antisym_part(a: np.ndarray) -> np.ndarray:
    """a^{a} = 1/2 (a - a^T) over the component indices (last two axes)."""
    return 0.5 * (a - np.swapaxes(a, -1, -2))
