"""The paper's linear elastostatics benchmark (Sec. 5.1.2) on the unit cube.

Orchestration only: every operator application, smoothing step, transfer and
solve runs in libhhg.so.  The mesh is the 6-macro Kuhn cube, whose refinement
at level l is the Freudenthal lattice of mesh size h = 2^-l; the paper's
384-tetrahedron mesh at its level l has the mesh size of level l + 2 here.

* Coefficient E = cos(m pi x y z) + 2 scales the form (1/(1+nu)) (eps, eps) +
  nu/((1+nu)(1-2nu)) (div, div), nu = 0.34 (eq. stressE).
* Load vector: "consistent": b = M I_h f, M the P1 mass matrix, whose rows
  on this lattice are h^3 (2/5 on the diagonal, 1/20 towards the 8
  neighbours along the six-element edges, 1/30 towards the 6 along the
  four-element edges); "lumped": b_i = f(x_i) h^3 (the integral of the hat
  function).
* Dirichlet data u* on the cube boundary: the solve is for the interior
  values w with A_uu w = b_u - A_ub g, where A_ub g is the apply of the same
  operator without Dirichlet nodes to the boundary values g.
* Error: the discrete L2 norm (h_L^3 sum over all nodes of |.|^2) of
  I u* - P v on the finest level L, P the P1 prolongation (exact for the
  nested P1 spaces), as in the paper.
"""
from __future__ import annotations

import sys
import time

import numpy as np


def _vec(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


_data = {}


def _pde_data(xyz, level, m):
    """E, u* and f at the nodes of one level (computed once per level and m)."""
    import workloads as W
    key = (level, m)
    if key not in _data:
        if len(_data) > 8:
            _data.clear()
        _data[key] = (W.elastostatics_modulus(xyz, m), W.elastostatics_solution(xyz),
                      W.elastostatics_force(xyz, m))
    return _data[key]


def consistent_load(xyz, F, level):
    """b = M I_h f at the slots (xyz, F: (n_slots, 3)); rows of nodes on the
    cube boundary are left at zero (they are Dirichlet rows)."""
    n = 1 << level
    I = np.rint(xyz * n).astype(np.int64)
    G = np.zeros((n + 1, n + 1, n + 1, 3))
    G[I[:, 0], I[:, 1], I[:, 2]] = F
    B = np.zeros_like(G)
    inner = (slice(1, n), slice(1, n), slice(1, n))
    B[inner] = 0.4 * G[inner]

    def shifted(d):
        return G[1 + d[0]:n + d[0], 1 + d[1]:n + d[1], 1 + d[2]:n + d[2]]
    six = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    four = [(1, 1, 0), (1, 0, 1), (0, 1, 1)]
    for d in six:
        B[inner] += (shifted(d) + shifted(tuple(-c for c in d))) / 20.0
    for d in four:
        B[inner] += (shifted(d) + shifted(tuple(-c for c in d))) / 30.0
    return B[I[:, 0], I[:, 1], I[:, 2]] / float(n) ** 3


def solve_level(level, m, corr="physical", iface="rowwise", method="cycle", op_method="scaled",
                load="consistent", rtol=1e-8, maxit=200, coarse=2, precision="f64", nu_inc=0,
                dev="cuda"):
    """Discrete solution on one level: (u_h [3, n_slots] with the boundary
    values, solve info, seconds of the solve).  precision: arithmetic of the
    V-cycles ("f64" or "f32"; residuals and updates stay FP64); nu_inc:
    extra smoothing steps per coarser level (the variable V-cycle)."""
    import torch
    import workloads as W
    from .hhg import Mesh, Multigrid
    mu, lam = W.eform_weights()
    mg = Multigrid(W.kuhn6(), level, coarse, mu1=mu, lam1=lam, corr=corr, iface=iface)
    neu = Mesh(W.kuhn6(), level, mu1=mu, lam1=lam, dirichlet="none", corr=corr, iface=iface)
    try:
        me = mg.meshes[-1]
        xyz = me.coords().T
        dirich = (_vec(me.flags(), dev) & 1) > 0
        E, U, F = _pde_data(xyz, level, m)
        k = _vec(E, dev)
        us = _vec(U.T, dev)
        g = torch.where(dirich[None, :], us, torch.zeros_like(us))
        h = 1.0 / (1 << level)
        f = _vec((consistent_load(xyz, F, level) if load == "consistent" else h ** 3 * F).T, dev)
        Ag = neu.apply_scaled(g, k) if op_method == "scaled" else neu.apply_onthefly(g, k)
        b = f - Ag
        b[:, dirich] = 0.0
        mg.setup_coefficient(k, method=op_method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, info = mg.solve(b, rtol=rtol, maxit=maxit, method=method, precision=precision,
                           nu_inc=nu_inc, raise_on_status=False)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        return w + g, info, secs
    finally:
        mg.close()
        neu.close()


class FineLevel:
    """Prolongation chain to the finest level and the interpolant of u* there."""

    def __init__(self, level, coarse=2, dev="cuda"):
        import workloads as W
        from .hhg import Multigrid
        mu, lam = W.eform_weights()
        # no Dirichlet nodes: the prolongation keeps the boundary values
        self.mg = Multigrid(W.kuhn6(), level, coarse, mu1=mu, lam1=lam, dirichlet="none")
        fm = self.mg.meshes[-1]
        xyz = fm.coords().T
        self.level = level
        self.owner = _vec((fm.flags() & 2) > 0, dev)
        self.u = _vec(W.elastostatics_solution(xyz).T, dev)
        self.h3 = (1.0 / (1 << level)) ** 3

    def error(self, u_h, level):
        import torch
        for q in range(level + 1, self.level + 1):
            u_h = self.mg.prolong(q, u_h)
        e = (self.u - u_h)[:, self.owner]
        return float(torch.sqrt(self.h3 * (e * e).sum()))

    def close(self):
        self.mg.close()


def benchmark(levels, finest, ms=(1, 2, 3, 8), variants=None, dev="cuda"):
    """Errors, convergence orders and solve iterations per (m, variant)."""
    variants = variants or {"physical": dict(corr="physical", op_method="scaled"),
                            "nodal": dict(corr="physical", op_method="onthefly"),
                            "unphysical": dict(corr="none", op_method="scaled")}
    fine = FineLevel(finest, dev=dev)
    out = {}
    try:
        for m in ms:
            for name, kw in variants.items():
                rows = []
                for lev in levels:
                    u_h, info, secs = solve_level(lev, m, dev=dev, **kw)
                    err = fine.error(u_h, lev)
                    print(f"elastostatics m={m} {name} level {lev}: error {err:.3e}, "
                          f"{info['iterations']} iterations, {secs:.3f} s", file=sys.stderr, flush=True)
                    eoc = (float(np.log2(rows[-1]["error"] / err)) if rows else None)
                    rows.append(dict(level=lev, error=err, eoc=None if eoc is None else round(eoc, 3),
                                     iterations=info["iterations"], status=info["status"],
                                     solve_seconds=round(secs, 4)))
                out[f"m{m}_{name}"] = rows
    finally:
        fine.close()
    return out
