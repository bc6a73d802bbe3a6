"""Learned 3x3 block smoother for flexible CG (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the test suite and the benchmark's CPU
baseline, never by the product path; shares no code with the HIP library.

The paper solves with multigrid and has no learned component; this module is
the plain FP64 definition of the learned preconditioner that sits beside the
block-Jacobi one, written out from its definition:

* Features of a node copy (one per macro holding the node): the coefficient
  k on the 15-point patch of the micro-mesh (the node and its 14 stencil
  neighbours, Sec. 2.4, Fig. subtypes_and_stencil), in the direction order
  me mw mse mnw tc bc ts bn mn ms tw be tse bnw.  A neighbour that is a
  Dirichlet node contributes 0, one outside the macro repeats the node's own
  value.  The 15 values are divided by their mean; the 16th feature is
  level / 8.  Features are rounded FP64 -> FP32 -> BF16 (nearest even).
* Network: h = relu(W1^T f + b1) (64 units, h rounded to BF16), o = W2^T h
  + b2 (9 outputs), with BF16 weights W1 (16x64), W2 (64x9) and FP32 biases.
  M = o as a row-major 3x3 matrix.
* Preconditioner block of a node: G = I + Mbar, P = G^T D^{-1} G, where D is
  the 3x3 diagonal block of the assembled operator and Mbar the mean of M
  over the node's copies.  M = 0 gives block Jacobi exactly; P is symmetric
  positive definite whenever G is invertible.
* Training sample: (f, r, e, S) with r, e the residual and error of an
  iterate of the plain solver at that node and S = t D^{-1}, r scaled by 1/t,
  t = trace(D)/3, and r, e divided by s = sqrt(|D^{-1} r|^2 + |e|^2).  Loss
  of a sample: |G^T S G r - e|^2, the error left by one smoothing step
  z = P r relative to the size of the error and of the block-Jacobi step
  (bounded for rough and for smooth errors alike), averaged over a batch.  Gradients pass the BF16 roundings straight through.
* Adam update of the FP32 master weights.
* Flexible CG (Polak-Ribiere beta), which reduces to preconditioned CG for a
  fixed symmetric positive definite preconditioner.

Parity: pinned by tests (central finite differences of the unrounded loss
against the analytic gradient; zero head gives the inverse diagonal blocks;
FCG equals PCG for a fixed SPD preconditioner; brute-force patch features on
a tiny mesh; BF16 rounding against hand-computed bit patterns).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

N_IN, N_HID, N_OUT = 16, 64, 9
N_PARAM = N_IN * N_HID + N_HID + N_HID * N_OUT + N_OUT

# stencil directions as (i, j, k) index offsets, paper's names
DIRS = np.array([(1, 0, 0), (-1, 0, 0), (1, -1, 0), (-1, 1, 0), (0, 0, 1), (0, 0, -1),
                 (0, -1, 1), (0, 1, -1), (0, 1, 0), (0, -1, 0), (-1, 0, 1), (1, 0, -1),
                 (1, -1, 1), (-1, 1, -1)], dtype=np.int64)


def bf16_round(x) -> np.ndarray:
    """FP64 -> FP32 (nearest even) -> BF16 (nearest even), returned as FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_ulp(x) -> np.ndarray:
    """Spacing of BF16 numbers at |x| (0 at x = 0)."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    safe = np.where(a > 0, a, 1.0)
    return np.where(a > 0, 2.0 ** (np.floor(np.log2(safe)) - 7), 0.0)


# ------------------------------------------------------------------ params

def unpack(w):
    """Flat parameter vector -> (W1 16x64, b1 64, W2 64x9, b2 9)."""
    w = np.asarray(w, dtype=np.float64)
    a = N_IN * N_HID
    b = a + N_HID
    c = b + N_HID * N_OUT
    return w[:a].reshape(N_IN, N_HID), w[a:b], w[b:c].reshape(N_HID, N_OUT), w[c:]


def pack(W1, b1, W2, b2) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2)])


def init_params(rng: np.random.Generator) -> np.ndarray:
    """He-uniform first layer, zero biases and zero second layer (the
    network starts as block Jacobi)."""
    lim = np.sqrt(6.0 / N_IN)
    W1 = rng.uniform(-lim, lim, size=(N_IN, N_HID)).astype(np.float32).astype(np.float64)
    return pack(W1, np.zeros(N_HID), np.zeros((N_HID, N_OUT)), np.zeros(N_OUT))


# ---------------------------------------------------------------- features

def macro_features(mesh, m: int, k: np.ndarray) -> np.ndarray:
    """Features (n_local, 16) of every local node of macro m (see module
    docstring), k given per distinct node."""
    n = 1 << int(mesh.levels[m])
    ijk = mesh.local_ijk[m].astype(np.int64)
    gid = mesh.gid[m]
    key = {tuple(v): q for q, v in enumerate(ijk.tolist())}
    vals = np.empty((ijk.shape[0], 15))
    kc = k[gid]
    vals[:, 0] = kc
    for d, off in enumerate(DIRS):
        nb = ijk + off
        inside = np.all(nb >= 0, axis=1) & (nb.sum(1) <= n)
        col = kc.copy()
        for q in np.nonzero(inside)[0]:
            g = gid[key[tuple(nb[q])]]
            col[q] = 0.0 if mesh.dirichlet[g] else k[g]
        vals[:, 1 + d] = col
    # the mean of the 15 patch values, from their correctly rounded sum
    mean = np.array([math.fsum(row) for row in vals]) / 15.0
    F = np.empty((ijk.shape[0], N_IN))
    F[:, :15] = vals / mean[:, None]
    F[:, 15] = n.bit_length() - 1
    F[:, 15] /= 8.0
    return bf16_round(F)


# ----------------------------------------------------------------- network

def forward(w, F, rounding=True):
    """Outputs o (n, 9) and the cache (z1, h, W1r, W2r) for backward."""
    W1, b1, W2, b2 = unpack(w)
    if rounding:
        W1, W2 = bf16_round(W1), bf16_round(W2)
        b1 = b1.astype(np.float32).astype(np.float64)
        b2 = b2.astype(np.float32).astype(np.float64)
    z1 = F @ W1 + b1
    h = np.maximum(z1, 0.0)
    if rounding:
        h = bf16_round(h)
    o = h @ W2 + b2
    return o, (z1, h, W1, W2)


def precond_blocks(o, Dinv):
    """P = (I + M)^T Dinv (I + M) per node; o (n, 9), Dinv (n, 3, 3)."""
    G = np.eye(3)[None] + o.reshape(-1, 3, 3)
    return np.einsum("nba,nbc,ncd->nad", G, Dinv, G)


def sym6_to_mat(s6):
    """(n, 6) xx yy zz xy xz yz -> (n, 3, 3)."""
    s6 = np.asarray(s6, dtype=np.float64)
    out = np.empty((s6.shape[0], 3, 3))
    out[:, 0, 0], out[:, 1, 1], out[:, 2, 2] = s6[:, 0], s6[:, 1], s6[:, 2]
    out[:, 0, 1] = out[:, 1, 0] = s6[:, 3]
    out[:, 0, 2] = out[:, 2, 0] = s6[:, 4]
    out[:, 1, 2] = out[:, 2, 1] = s6[:, 5]
    return out


def loss_and_grad(w, F, r, e, S6, rounding=True):
    """Mean sample loss |G^T S G r - e|^2 and its gradient (flat, N_PARAM)."""
    B = F.shape[0]
    S = sym6_to_mat(S6)
    o, (z1, h, W1r, W2r) = forward(w, F, rounding)
    G = np.eye(3)[None] + o.reshape(-1, 3, 3)
    u = np.einsum("nab,nb->na", G, r)          # G r
    v = np.einsum("nab,nb->na", S, u)          # S G r
    z = np.einsum("nba,nb->na", G, v)          # G^T S G r
    d = z - e
    loss = np.einsum("na,na->n", d, d).mean()
    # dl/dz = 2 d / B; z = G^T v  ->  dG += v d^T, dv = G dz
    dz = 2.0 * d / B
    dG = np.einsum("na,nb->nab", v, dz)
    dv = np.einsum("nab,nb->na", G, dz)
    du = np.einsum("nba,nb->na", S, dv)        # S symmetric
    dG += np.einsum("na,nb->nab", du, r)       # u = G r
    d2 = dG.reshape(B, N_OUT)
    gW2 = h.T @ d2
    gb2 = d2.sum(0)
    dh = d2 @ W2r.T
    dz1 = dh * (z1 > 0.0)
    gW1 = F.T @ dz1
    gb1 = dz1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2)


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------- preconditioner matrix

def diag_blocks(A: sp.spmatrix, nodes) -> np.ndarray:
    """3x3 diagonal blocks of A (dofs 3 node + component) at the given nodes."""
    A = A.tocsr()
    nodes = np.asarray(nodes)
    D = np.empty((nodes.shape[0], 3, 3))
    for a in range(3):
        for c in range(3):
            D[:, a, c] = A[3 * nodes + a, 3 * nodes + c].A1
    return D


def learned_blocks(mesh, k, w, A) -> np.ndarray:
    """P (n_nodes, 3, 3): G^T D^{-1} G with M averaged over the node's copies,
    zero at Dirichlet nodes.  A is the full (unreduced) operator matrix."""
    msum = np.zeros((mesh.n_nodes, 9))
    cnt = np.zeros(mesh.n_nodes)
    for m in range(mesh.n_macro):
        o, _ = forward(w, macro_features(mesh, m, k))
        np.add.at(msum, mesh.gid[m], o)
        np.add.at(cnt, mesh.gid[m], 1.0)
    mbar = msum / cnt[:, None]
    P = np.zeros((mesh.n_nodes, 3, 3))
    u = mesh.unknown
    Dinv = np.linalg.inv(diag_blocks(A, u))
    P[u] = precond_blocks(mbar[u], Dinv)
    return P


def block_matrix(P_nodes: np.ndarray, nodes) -> sp.csr_matrix:
    """Block-diagonal sparse matrix over the dofs of ``nodes`` (in order)."""
    n = len(nodes)
    blocks = P_nodes[np.asarray(nodes)]
    rows = (np.arange(n)[:, None, None] * 3 + np.arange(3)[None, :, None]).repeat(3, axis=2)
    cols = (np.arange(n)[:, None, None] * 3 + np.arange(3)[None, None, :]).repeat(3, axis=1)
    return sp.csr_matrix((blocks.ravel(), (rows.ravel(), cols.ravel())), shape=(3 * n, 3 * n))


# -------------------------------------------------------------------- FCG

def fcg(A, b, Pmat, x0=None, rtol=1e-8, maxiter=100000):
    """Flexible CG with the Polak-Ribiere beta = (z_new, r_new - r_old) /
    (z_old, r_old); stops at ||b - A x|| <= rtol ||b||.  Returns (x, iters)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bn = np.linalg.norm(b)
    z = Pmat @ r
    p = z.copy()
    rho = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * bn and it < maxiter:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r_new = r - alpha * q
        z = Pmat @ r_new
        rho_new = r_new @ z
        beta = (z @ (r_new - r)) / rho
        p = z + beta * p
        r, rho = r_new, rho_new
        it += 1
    return x, it


def pcg(A, b, Pmat, x0=None, rtol=1e-8, maxiter=100000):
    """Textbook preconditioned CG (Fletcher-Reeves beta = rho_new / rho)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bn = np.linalg.norm(b)
    z = Pmat @ r
    p = z.copy()
    rho = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * bn and it < maxiter:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r = r - alpha * q
        z = Pmat @ r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it


# ------------------------------------------------------------------ samples

def make_samples(F, r, e, D):
    """Training records from node values: features F (n, 16), residual r and
    error e (n, 3) of a solver iterate, diagonal blocks D (n, 3, 3).
    Returns (F, r', e', S6) with t = trace(D)/3, S = t D^{-1},
    s = sqrt(|D^{-1} r|^2 + |e|^2), r' = r / (t s), e' = e / s."""
    t = np.trace(D, axis1=1, axis2=2) / 3.0
    Dinv = np.linalg.inv(D)
    S = t[:, None, None] * Dinv
    s = np.sqrt(np.sum(np.einsum("nab,nb->na", Dinv, r) ** 2, axis=1) + np.sum(e * e, axis=1))
    rr = r / (t * s)[:, None]
    ee = e / s[:, None]
    S6 = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]], axis=1)
    return F, rr, ee, S6
