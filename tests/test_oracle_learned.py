"""Pins of the learned-smoother oracle (no GPU): BF16 rounding bit patterns,
brute-force patch features, finite-difference gradients, the zero-head
special case (block Jacobi), the sample normalisation, Adam's sign-descent
limit and FCG = PCG for a fixed SPD preconditioner."""
import numpy as np
import pytest

import workloads as W
from oracle import learned as LN
from oracle import operators as O
from oracle import solvers as S
from oracle.mesh import MacroMesh


def test_bf16_round_bit_patterns():
    one = 1.0
    cases = [
        (1.0, 1.0),
        (one + 2.0 ** -8, 1.0),                              # halfway, even stays
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),              # halfway, odd rounds up
        (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),     # above halfway
        (-(one + 2.0 ** -8 + 2.0 ** -20), -(one + 2.0 ** -7)),
        (one + 2.0 ** -8 + 2.0 ** -30, 1.0),                 # FP32 step first: back to halfway
        (3.0e38, 2.0 ** 127 * (1 + 98 / 128)),                # 3e38 / 2^127 = 1.7632..., 0.7632 * 128 = 97.7
        (0.0, 0.0),
    ]
    for x, want in cases:
        got = LN.bf16_round(np.array([x]))[0]
        assert got == want, (x, got, want)
    # idempotent, at most half a BF16 ulp away
    x = np.random.default_rng(0).normal(size=1000) * 10
    y = LN.bf16_round(x)
    assert np.array_equal(LN.bf16_round(y), y)
    ulp = 2.0 ** (np.floor(np.log2(np.abs(x))) - 7)
    assert np.all(np.abs(y - x) <= 0.5 * ulp * (1 + 1e-9))


def test_features_brute_force_by_coordinates():
    """Patch values found geometrically (neighbour position = node position
    plus the direction mapped by the macro's edge vectors) on a kuhn6 mesh."""
    mesh = MacroMesh(W.kuhn6(), 2)
    k = W.exp_fourier_coefficient(mesh.xyz, W.rng_for(5, 1), 8, 1.0)
    for m in range(mesh.n_macro):
        F = LN.macro_features(mesh, m, k)
        n = 4
        E = (mesh.verts[m, 1:] - mesh.verts[m, 0]) / n
        xyz_m = mesh.local_xyz[m]
        ijk = mesh.local_ijk[m]
        for q in range(xyz_m.shape[0]):
            g = mesh.gid[m][q]
            vals = [k[g]]
            for off in LN.DIRS:
                p = xyz_m[q] + off @ E
                dist = np.linalg.norm(xyz_m - p, axis=1)
                hit = np.nonzero(dist < 1e-12)[0]
                if hit.size == 0:
                    vals.append(k[g])
                else:
                    gg = mesh.gid[m][hit[0]]
                    vals.append(0.0 if mesh.dirichlet[gg] else k[gg])
            vals = np.array(vals)
            want = LN.bf16_round(np.concatenate([vals / vals.mean(), [2 / 8]]))
            # the mean's last bit may depend on the summation order, which can
            # move a BF16 rounding by one unit
            assert np.all(np.abs(F[q] - want) <= LN.bf16_ulp(want)), (m, q, ijk[q])


def _random_batch(B=40, seed=3):
    rng = np.random.default_rng(seed)
    F = LN.bf16_round(rng.uniform(0, 2, size=(B, 16)))
    r = rng.normal(size=(B, 3))
    e = rng.normal(size=(B, 3))
    A = rng.normal(size=(B, 3, 3))
    S6 = np.einsum("nab,ncb->nac", A, A) + 0.5 * np.eye(3)
    S6 = np.stack([S6[:, 0, 0], S6[:, 1, 1], S6[:, 2, 2], S6[:, 0, 1], S6[:, 0, 2], S6[:, 1, 2]], 1)
    w = LN.init_params(rng)
    w[LN.N_IN * LN.N_HID:] = rng.normal(scale=0.3, size=LN.N_PARAM - LN.N_IN * LN.N_HID)
    return w, F, r, e, S6


def test_gradient_central_differences():
    w, F, r, e, S6 = _random_batch()
    loss, g = LN.loss_and_grad(w, F, r, e, S6, rounding=False)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(LN.N_IN * LN.N_HID, 30, replace=False),
                          np.arange(LN.N_IN * LN.N_HID, LN.N_PARAM)])
    h = 1e-4
    tol_round = 1e-15 * loss / h          # cancellation in the difference quotient
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (LN.loss_and_grad(wp, F, r, e, S6, rounding=False)[0] -
              LN.loss_and_grad(wm, F, r, e, S6, rounding=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + tol_round, (i, fd, g[i])


def test_zero_head_is_block_jacobi_and_sample_loss():
    mesh = MacroMesh(W.kuhn6(), 2)
    mu, lam = W.eform_weights()
    op = dict(mu1=mu, lam1=lam)
    k = W.exp_fourier_coefficient(mesh.xyz, W.rng_for(5, 2), 8, 1.0)
    A = O.operator_matrix(mesh, k, op)
    w = LN.init_params(np.random.default_rng(1))       # second layer zero
    P = LN.learned_blocks(mesh, k, w, A)
    Auu, dof = S.reduced_system(mesh, k, op)
    BJ = S.block_jacobi_inverse(Auu).toarray()
    Pm = LN.block_matrix(P, mesh.unknown).toarray()
    assert np.allclose(Pm, BJ, rtol=1e-13, atol=1e-13 * np.abs(BJ).max())
    # loss of a sample with M = 0 is |D^{-1} r - e|^2 / (|D^{-1} r|^2 + |e|^2)
    rng = np.random.default_rng(2)
    u = mesh.unknown
    D = LN.diag_blocks(A, u)
    r = rng.normal(size=(u.size, 3))
    e = rng.normal(size=(u.size, 3))
    F = np.concatenate([LN.macro_features(mesh, 0, k)] * 10)[: u.size]
    Fs, rs, es, S6 = LN.make_samples(F, r, e, D)
    loss, _ = LN.loss_and_grad(w, Fs, rs, es, S6)
    Dr = np.einsum("nab,nb->na", np.linalg.inv(D), r)
    want = np.mean(np.sum((Dr - e) ** 2, 1) / (np.sum(Dr ** 2, 1) + np.sum(e ** 2, 1)))
    assert abs(loss - want) <= 1e-12 * want


def test_precond_block_by_hand():
    """One node with M = e_x e_y^T (o row-major: o[1] = 1) and D = diag(1, 2, 4):
    G = I + M = [[1,1,0],[0,1,0],[0,0,1]], D^-1 G = [[1,1,0],[0,1/2,0],[0,0,1/4]],
    P = G^T D^-1 G = [[1,1,0],[1,3/2,0],[0,0,1/4]].  G D^-1 G^T would give
    [[3/2,1/2,0],[1/2,1/2,0],[0,0,1/4]], and a column-major M the same with
    rows and columns 0, 1 swapped in the role of G."""
    o = np.zeros((1, 9))
    o[0, 1] = 1.0
    Dinv = np.diag([1.0, 0.5, 0.25])[None]
    P = LN.precond_blocks(o, Dinv)
    np.testing.assert_array_equal(P[0], [[1.0, 1.0, 0.0], [1.0, 1.5, 0.0], [0.0, 0.0, 0.25]])
    # a non-symmetric full M against a hand-expanded product
    o2 = np.array([[0.5, -1.0, 2.0, 0.0, 1.0, 0.25, -0.5, 3.0, 0.0]])
    D = np.array([[2.0, 1.0, 0.0], [1.0, 3.0, 1.0], [0.0, 1.0, 4.0]])
    G = np.array([[1.5, -1.0, 2.0], [0.0, 2.0, 0.25], [-0.5, 3.0, 1.0]])
    Di = np.linalg.inv(D)
    want = np.zeros((3, 3))
    for a in range(3):
        for d in range(3):
            want[a, d] = sum(G[b, a] * Di[b, c] * G[c, d] for b in range(3) for c in range(3))
    np.testing.assert_allclose(LN.precond_blocks(o2, Di[None])[0], want, rtol=1e-14, atol=1e-14)


def test_adam_sign_descent_limit():
    """beta1 = beta2 = 0: the step is lr * g / (|g| + eps) per entry."""
    rng = np.random.default_rng(4)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m, v = LN.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=0.01, beta1=0.0, beta2=0.0,
                            eps=0.0)
    assert np.allclose(w1, w - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.array_equal(m, g) and np.array_equal(v, g * g)


def test_fcg_equals_pcg_for_fixed_spd_preconditioner():
    mesh = MacroMesh(W.kuhn6(), 3)
    mu, lam = W.eform_weights()
    op = dict(mu1=mu, lam1=lam)
    k = W.exp_fourier_coefficient(mesh.xyz, W.rng_for(5, 3), 8, 1.0)
    Auu, dof = S.reduced_system(mesh, k, op)
    M = S.block_jacobi_inverse(Auu)
    b = np.random.default_rng(6).uniform(-1, 1, size=Auu.shape[0])
    x1, i1 = LN.fcg(Auu, b, M, rtol=1e-10)
    x2, i2 = LN.pcg(Auu, b, M, rtol=1e-10)
    xs = S.direct_solve(Auu, b)
    assert abs(i1 - i2) <= 1
    assert np.linalg.norm(x1 - xs) <= 1e-8 * np.linalg.norm(xs)
    assert np.linalg.norm(x2 - xs) <= 1e-8 * np.linalg.norm(xs)
    # and the flexible variant still converges with a non-symmetric one
    Mn = (M @ (sp_eye(Auu.shape[0]) + 0.05 * sp_rand(Auu.shape[0]))).tocsr()
    x3, i3 = LN.fcg(Auu, b, Mn, rtol=1e-10, maxiter=5000)
    assert np.linalg.norm(Auu @ x3 - b) <= 1e-10 * np.linalg.norm(b) and i3 < 5000


def sp_eye(n):
    import scipy.sparse as sp
    return sp.eye(n, format="csr")


def sp_rand(n):
    import scipy.sparse as sp
    return sp.diags(np.random.default_rng(7).uniform(-1, 1, size=n), format="csr")
