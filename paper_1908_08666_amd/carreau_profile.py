"""Physical, nodal-integration and unphysical scaling in the non-linear
Carreau flow (Sec. 5.2.2, Fig. stokes_profile), on the 6-macro unit cube.

Orchestration only: the fixed-point iterations, solves and viscosity
updates run in libhhg.so.  The paper's channel geometry is not available, so
the flow here is driven in the no-slip unit cube by the body force
f = (0, 0, F sin(2 pi x)) (its curl is non-zero, so it is not absorbed by
the pressure), with the paper's dimensionless Carreau parameters.  The load
vector is f(x_i) h^3 (the hat-function integral of an interior node of the
Kuhn lattice).  Viscosity and velocity magnitude are sampled on the line
y = z = 1/2 and compared with nodal integration.
"""
from __future__ import annotations

import numpy as np

PAPER_LAW = dict(eta0=140.764, eta_inf=1.0, kappa=212.2, r=-0.325)


def profiles(level, force=1000.0, law=None, coarse=2, rtol=1e-6, maxit=3000, max_picard=400,
             dev="cuda"):
    """Picard runs for the three operators; returns the line samples and the
    deviations from nodal integration: largest (relative to its maxima) and
    in the 2-norm over the line (relative to its norm).  The largest
    viscosity deviation sits at the stagnation points, where mu is close to
    eta0 and most sensitive to the strain rate."""
    import torch
    import workloads as W
    from .hhg import Multigrid
    law = dict(PAPER_LAW if law is None else law)
    variants = {"physical": dict(corr="physical", method="scaled"),
                "nodal": dict(corr="physical", method="onthefly"),
                "unphysical": dict(corr="none", method="scaled")}
    out = dict(level=level, force=force, law=law, line="y = z = 1/2", runs={})
    for name, v in variants.items():
        mg = Multigrid(W.kuhn6(), level, coarse, mu1=1.0, corr=v["corr"])
        try:
            fm = mg.meshes[-1]
            xyz = fm.coords().T
            flags = fm.flags()
            h3 = (1.0 / (1 << level)) ** 3
            f = np.zeros((3, fm.n_nodes))
            f[2] = force * np.sin(2 * np.pi * xyz[:, 0]) * h3
            f[:, (flags & 1) > 0] = 0.0
            ft = torch.from_numpy(f).to(dev)
            u, p, mu, info = mg.stokes_picard(ft, **law, method=v["method"], rtol=rtol, maxit=maxit,
                                              max_picard=max_picard)
            torch.cuda.synchronize()
            on = np.nonzero((np.abs(xyz[:, 1] - 0.5) < 1e-12) & (np.abs(xyz[:, 2] - 0.5) < 1e-12))[0]
            xs, first = np.unique(xyz[on, 0], return_index=True)
            sl = on[first]
            un = torch.linalg.vector_norm(u, dim=0).cpu().numpy()
            out["runs"][name] = dict(x=xs.tolist(), mu=mu.cpu().numpy()[sl].tolist(),
                                     speed=un[sl].tolist(), picard=info["picard"],
                                     final_iterations=info["final_iterations"], status=info["status"],
                                     seconds=round(info["seconds"], 4),
                                     mu_range=[float(mu.min()), float(mu.max())])
        finally:
            mg.close()
    ref = out["runs"]["nodal"]
    for name in ("physical", "unphysical"):
        r = out["runs"][name]
        dmu, dsp = np.subtract(r["mu"], ref["mu"]), np.subtract(r["speed"], ref["speed"])
        out[f"{name}_vs_nodal"] = dict(
            mu=float(np.abs(dmu).max() / np.max(ref["mu"])),
            speed=float(np.abs(dsp).max() / np.max(ref["speed"])),
            mu_l2=float(np.linalg.norm(dmu) / np.linalg.norm(ref["mu"])),
            speed_l2=float(np.linalg.norm(dsp) / np.linalg.norm(ref["speed"])))
    return out
