"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds only input generation: macro meshes (vertex lists), nodal
coefficient fields and random vectors.  It contains none of the stencil-scaling
arithmetic, so both the CPU oracle and the GPU library can consume its outputs
without sharing any of the method's code.

Workloads (the paper's setting of vector-valued P1 elasticity / generalized
Newtonian operators on uniformly refined macro-tetrahedra, Sec. 2 and Sec. 5):

* ``unit_tet``   one reference macro-tet, level 4 (969 nodes), k = 1 + 0.5
                 sin(2 pi x) sin(2 pi y) sin(2 pi z), Lame mu = 1, lambda = k.
* ``kuhn6``      unit cube cut into 6 macro-tets along the main diagonal
                 (vertex order 0, e_s1, e_s1+e_s2, 1 for every permutation s),
                 level 7, k = exp(g) with g a 16-mode smooth random field of
                 amplitude 1; paper's E-form elasticity with nu = 0.34 (Sec. 5.1.2).
* ``cube24``     unit cube: every face cut into 4 triangles through its centre,
                 every triangle joined to the cube centre (24 congruent macros),
                 level 7, Carreau viscosity of a seeded smooth velocity field.
* ``batch256``   256 independent unit macro-tets, levels uniform in 3..6, each
                 with its own Fourier coefficient field.
* ``elastostatics_*``  the paper's linear elastostatics benchmark (Sec. 5.1.2):
                 Young's modulus E = cos(m pi x y z) + 2, manufactured solution
                 u*, body force f = -div sigma(u*) (PDE data, derived exactly
                 by automatic differentiation).
"""
from __future__ import annotations

import itertools

import numpy as np

SEED_BASE = 190808666


def rng_for(config_id: int, salt: int = 0) -> np.random.Generator:
    """Seeded generator for a workload id (config 1..5) and a salt."""
    return np.random.default_rng([SEED_BASE + config_id, salt])


# ---------------------------------------------------------------- macro meshes

def unit_tet() -> np.ndarray:
    """Reference macro-tet (0,0,0),(1,0,0),(0,1,0),(0,0,1); shape (1,4,3)."""
    return np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0],
                      [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]])


def kuhn6() -> np.ndarray:
    """Unit cube split into 6 tets sharing the main diagonal; shape (6,4,3).

    Vertex order (0, e_s1, e_s1 + e_s2, (1,1,1)) for each permutation s, so
    every macro's micro-lattice is the same Freudenthal lattice of the cube.
    """
    eye = np.eye(3)
    out = []
    for s in itertools.permutations(range(3)):
        v1 = eye[s[0]]
        v2 = v1 + eye[s[1]]
        out.append([np.zeros(3), v1, v2, np.ones(3)])
    return np.array(out, dtype=np.float64)


def cube24() -> np.ndarray:
    """Unit cube: each face split into 4 triangles through the face centre,
    each triangle joined to the cube centre; shape (24,4,3).

    Vertex order (cube centre, face centre, corner a, corner b) with corners
    a, b consecutive around the face.
    """
    c = np.full(3, 0.5)
    out = []
    for axis in range(3):
        for side in (0.0, 1.0):
            fc = np.full(3, 0.5)
            fc[axis] = side
            u, w = [a for a in range(3) if a != axis]
            ring = []
            for du, dw in ((0, 0), (1, 0), (1, 1), (0, 1)):
                p = np.zeros(3)
                p[axis] = side
                p[u] = du
                p[w] = dw
                ring.append(p)
            for q in range(4):
                out.append([c, fc, ring[q], ring[(q + 1) % 4]])
    return np.array(out, dtype=np.float64)


def twod_mesh(name: str) -> np.ndarray:
    """2-D macro triangulations (M, 3, 2): "triangle" (the unit right
    triangle), "square" (the unit square cut along its anti-diagonal) and
    "cross" (the unit square cut into four triangles through its centre,
    so that one vertex is shared by four macros)."""
    if name == "triangle":
        return np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    if name == "square":
        return np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]],
                         [[1.0, 1.0], [0.0, 1.0], [1.0, 0.0]]])
    if name == "cross":
        c = [0.5, 0.5]
        return np.array([[c, [0.0, 0.0], [1.0, 0.0]], [c, [1.0, 0.0], [1.0, 1.0]],
                         [c, [1.0, 1.0], [0.0, 1.0]], [c, [0.0, 1.0], [0.0, 0.0]]])
    raise ValueError(name)


def batch_levels(n_problems: int = 256, lo: int = 3, hi: int = 6,
                 config_id: int = 4) -> np.ndarray:
    """Levels of the independent batched problems, uniform in lo..hi."""
    return rng_for(config_id, 1).integers(lo, hi + 1, size=n_problems).astype(np.int32)


def batch_field_params(n_problems: int = 256, config_id: int = 4):
    """Per-problem (n_modes, amplitude) for the batched workload."""
    r = rng_for(config_id, 2)
    modes = r.integers(4, 33, size=n_problems)
    amps = r.uniform(0.5, 2.0, size=n_problems)
    return modes, amps


def batch_coefficients(local_xyz, config_id: int = 4) -> list:
    """One coefficient field per independent problem: k = exp(g_p) with g_p a
    Fourier field of that problem's mode count and amplitude
    (``batch_field_params``), drawn from its own seed; ``local_xyz`` lists the
    node coordinates of each problem."""
    modes, amps = batch_field_params(len(local_xyz), config_id)
    return [exp_fourier_coefficient(xyz, rng_for(config_id, 1000 + p), int(modes[p]), float(amps[p]))
            for p, xyz in enumerate(local_xyz)]


# -------------------------------------------------------------- nodal fields

def sine_coefficient(xyz: np.ndarray) -> np.ndarray:
    """k(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z) at points (N,3)."""
    s = np.sin(2.0 * np.pi * xyz)
    return 1.0 + 0.5 * s[:, 0] * s[:, 1] * s[:, 2]


def affine_coefficient(xyz: np.ndarray, a0=1.5, grad=(0.3, -0.2, 0.45)) -> np.ndarray:
    """A globally affine positive coefficient a0 + grad . x."""
    return a0 + xyz @ np.asarray(grad, dtype=np.float64)


def fourier_modes(rng: np.random.Generator, n_modes: int, kmax: int = 4):
    """Draw n_modes wave vectors in {-kmax..kmax}^3 \\ {0}, phases, amplitudes."""
    kv = []
    while len(kv) < n_modes:
        v = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(v != 0):
            kv.append(v)
    kv = np.array(kv, dtype=np.float64)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    amp = rng.uniform(-1.0, 1.0, size=n_modes)
    return kv, phase, amp


def fourier_field(xyz: np.ndarray, rng: np.random.Generator, n_modes: int,
                  amplitude: float) -> np.ndarray:
    """Smooth random field g = sum_m a_m cos(2 pi kappa_m . x + phi_m), rescaled
    so that max |g| over the given points equals ``amplitude``."""
    kv, phase, amp = fourier_modes(rng, n_modes)
    g = np.cos(2.0 * np.pi * xyz @ kv.T + phase) @ amp
    m = np.max(np.abs(g))
    return g * (amplitude / m) if m > 0 else g


def exp_fourier_coefficient(xyz: np.ndarray, rng: np.random.Generator,
                            n_modes: int = 16, amplitude: float = 1.0) -> np.ndarray:
    """k = exp(g) with g a Fourier field of the given amplitude (k in [e^-A, e^A])."""
    return np.exp(fourier_field(xyz, rng, n_modes, amplitude))


def velocity_modes(rng: np.random.Generator, n_modes: int = 8, kmax: int = 3):
    kv = []
    while len(kv) < n_modes:
        v = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(v != 0):
            kv.append(v)
    kv = np.array(kv, dtype=np.float64)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    b = rng.uniform(-1.0, 1.0, size=(n_modes, 3))
    return kv, phase, b


def velocity_field(xyz: np.ndarray, rng: np.random.Generator, scale: float,
                   n_modes: int = 8) -> np.ndarray:
    """Smooth velocity u(x) = A sum_m b_m sin(2 pi kappa_m . x + phi_m); (N,3)."""
    kv, phase, b = velocity_modes(rng, n_modes)
    return scale * (np.sin(2.0 * np.pi * xyz @ kv.T + phase) @ b)


def velocity_gradient(xyz: np.ndarray, rng: np.random.Generator, scale: float,
                      n_modes: int = 8) -> np.ndarray:
    """Analytic gradient G[n, c, d] = d u_c / d x_d of ``velocity_field`` drawn
    from an identically seeded generator."""
    kv, phase, b = velocity_modes(rng, n_modes)
    cosv = np.cos(2.0 * np.pi * xyz @ kv.T + phase)          # (N, M)
    return scale * 2.0 * np.pi * np.einsum('nm,mc,md->ncd', cosv, b, kv)


def consistent_uniform(xyz: np.ndarray, owner: np.ndarray, rng: np.random.Generator,
                       ncomp: int = 3, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """U(lo, hi) values drawn once per distinct node (the slots flagged in
    ``owner``) and copied to every slot at the same position; (ncomp, n)."""
    from scipy.spatial import cKDTree
    owners = np.nonzero(owner)[0]
    _, idx = cKDTree(xyz[owners]).query(xyz)
    vals = rng.uniform(lo, hi, size=(ncomp, owners.shape[0]))
    return np.ascontiguousarray(vals[:, idx])


def uniform_vector(n: int, rng: np.random.Generator) -> np.ndarray:
    """Entries U(-1, 1), float64."""
    return rng.uniform(-1.0, 1.0, size=n)


def localized_velocity_field(xyz: np.ndarray, rng: np.random.Generator, scale: float,
                             width: float = 0.12, n_modes: int = 8) -> np.ndarray:
    """Smooth velocity concentrated around a seeded centre c in the middle of
    the unit cube: exp(-|x - c|^2 / (2 width^2)) times ``velocity_field``.
    Its strain rate spans many orders of magnitude across the cube, so the
    Carreau viscosity sweeps most of the range eta_inf .. eta0; (N, 3)."""
    c = rng.uniform(0.35, 0.65, size=3)
    env = np.exp(-np.sum((xyz - c) ** 2, axis=1) / (2.0 * width * width))
    return env[:, None] * velocity_field(xyz, rng, scale, n_modes)


def smoother_init_weights(rng: np.random.Generator) -> np.ndarray:
    """Initial parameters of the 16-64-9 smoother network as one FP32 vector
    (W1 [16][64] row-major, b1, W2 [64][9], b2): W1 He-uniform, everything
    else zero, so the untrained network is block Jacobi."""
    lim = np.sqrt(6.0 / 16.0)
    w = np.zeros(16 * 64 + 64 + 64 * 9 + 9, dtype=np.float32)
    w[:16 * 64] = rng.uniform(-lim, lim, size=16 * 64).astype(np.float32)
    return w


# ------------------------------------------------------- material constants

def eform_weights(nu: float = 0.34):
    """Paper's single-coefficient elasticity form (Sec. 5.1.2): E scales
    (1/(1+nu)) (eps, eps) + nu/((1+nu)(1-2nu)) (div, div).

    Returned as (mu, lam) with the form written 2 mu (eps, eps) + lam (div, div).
    """
    return 1.0 / (2.0 * (1.0 + nu)), nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


CARREAU_DEFAULT = dict(eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25)


# ------------------------------------------------ linear elastostatics benchmark
def elastostatics_modulus(xyz: np.ndarray, m: int) -> np.ndarray:
    """Young's modulus E(x, y, z) = cos(m pi x y z) + 2 (Sec. 5.1.2)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.cos(m * np.pi * x * y * z) + 2.0


def _u_star_t(X):
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    d = x * y * z + 1.0
    import torch
    return torch.stack([(x ** 3 * y + z ** 2) / d, (x ** 4 * y + 2.0 * z) / d,
                        (3.0 * x + y * z ** 3) / d], dim=1)


def elastostatics_solution(xyz: np.ndarray) -> np.ndarray:
    """Manufactured solution u*(x, y, z) of Sec. 5.1.2, (n, 3)."""
    import torch
    return _u_star_t(torch.from_numpy(np.asarray(xyz, dtype=np.float64))).numpy()


def elastostatics_force(xyz: np.ndarray, m: int, nu: float = 0.34, chunk: int = 1 << 18) -> np.ndarray:
    """Body force f = -div sigma(u*) with sigma = E (eps/(1+nu) +
    nu/((1+nu)(1-2nu)) tr(eps) I) (eq. stressE), (n, 3).  Derivatives are
    taken by automatic differentiation in FP64 (exact up to rounding)."""
    import torch
    a = 1.0 / (1.0 + nu)
    b = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    out = np.empty((xyz.shape[0], 3))
    for s in range(0, xyz.shape[0], chunk):
        X = torch.tensor(np.asarray(xyz[s:s + chunk], dtype=np.float64), requires_grad=True)
        u = _u_star_t(X)
        # grad u: G[:, c, d] = d u_c / d x_d
        G = torch.stack([torch.autograd.grad(u[:, c].sum(), X, create_graph=True)[0] for c in range(3)], dim=1)
        eps = 0.5 * (G + G.transpose(1, 2))
        tr = eps[:, 0, 0] + eps[:, 1, 1] + eps[:, 2, 2]
        E = torch.cos(m * np.pi * X[:, 0] * X[:, 1] * X[:, 2]) + 2.0
        sig = E[:, None, None] * (a * eps + b * tr[:, None, None] * torch.eye(3, dtype=X.dtype))
        f = torch.zeros((X.shape[0], 3), dtype=X.dtype)
        for c in range(3):
            for d in range(3):
                g = torch.autograd.grad(sig[:, c, d].sum(), X, retain_graph=True)[0]
                f[:, c] -= g[:, d]
        out[s:s + chunk] = f.detach().numpy()
    return out

