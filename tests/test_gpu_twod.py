"""GPU parity of the 2-D variant (Sec. 2, Sec. 2.3) against the 2-D oracle:
scaled (physical, unphysical, edge-mean khat) and nodal-integration applies
on one, two and four macro triangles under the three interface rules, FP64
and FP32, and sampled rows at a large level."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads as W
from oracle import twod as T2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)
MIXED = dict(mu0=1.0, lam1=1.0)
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def _s2n(lib, orc):
    d, idx = cKDTree(orc.xy).query(lib.coords().T)
    assert d.max() < 1e-9
    return idx


def _run(lib, s2n, x, k, dtype, method):
    xt = torch.from_numpy(np.ascontiguousarray(x[s2n].T)).to("cuda", dtype)
    kt = torch.from_numpy(k[s2n]).to("cuda", dtype)
    y = lib.apply_scaled(xt, kt) if method == "scaled" else lib.apply_onthefly(xt, kt)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _check(lib, orc, x, k, op, dtype, method, **kw):
    s2n = _s2n(lib, orc)
    y = _run(lib, s2n, x, k, dtype, method)
    yn = np.full((orc.n_nodes, 2), np.nan)
    yn[s2n] = y.T
    assert np.array_equal(yn[s2n], y.T), "copies of a node differ"
    if dtype == torch.float32:
        x, k = x.astype(np.float32).astype(np.float64), k.astype(np.float32).astype(np.float64)
    ref = T2.apply(orc, k, op, x, method="scaled" if method == "scaled" else "nodal", **kw)
    u = orc.unknown
    assert np.all(yn[orc.dirichlet] == 0)
    err = np.linalg.norm(yn[u] - ref[u]) / np.linalg.norm(ref[u])
    print(f"  {method} {dtype} {kw}: rel err {err:.2e}", flush=True)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,level", [("triangle", 4), ("square", 4), ("cross", 3)])
@pytest.mark.parametrize("iface", ["symmetric", "rowwise", "zerosum"])
def test_apply_matches_oracle(name, level, iface, dtype):
    from paper_1908_08666_amd.twod import Mesh2D
    orc = T2.Mesh2D(W.twod_mesh(name), level)
    lib = Mesh2D(W.twod_mesh(name), level, **EFORM, iface=iface)
    rng = np.random.default_rng(11)
    k = np.exp(W.fourier_field(np.column_stack([orc.xy, np.zeros(orc.n_nodes)]), rng, 8, 1.0))
    x = rng.uniform(-1, 1, (orc.n_nodes, 2))
    _check(lib, orc, x, k, EFORM, dtype, "scaled", iface=iface)
    _check(lib, orc, x, k, EFORM, dtype, "onthefly")
    lib.close()


@pytest.mark.parametrize("variant", [dict(corr="none"), dict(khat="edge"), dict()])
def test_variants_and_constant_part(variant):
    """Unphysical scaling, the edge-mean khat, and a form with an unscaled
    part (mu = 1, lambda = k), without Dirichlet nodes (every macro edge a
    boundary of listed rows)."""
    from paper_1908_08666_amd.twod import Mesh2D
    orc = T2.Mesh2D(W.twod_mesh("square"), 4, dirichlet="none")
    lib = Mesh2D(W.twod_mesh("square"), 4, **MIXED, dirichlet="none", **variant)
    rng = np.random.default_rng(12)
    k = 1.5 + np.sin(3 * orc.xy[:, 0]) * np.cos(2 * orc.xy[:, 1])
    x = rng.uniform(-1, 1, (orc.n_nodes, 2))
    if variant.get("khat") == "edge":
        # the oracle knows only the patch mean; for affine k the two agree
        k = 1.5 + 0.3 * orc.xy[:, 0] - 0.2 * orc.xy[:, 1]
        _check(lib, orc, x, k, MIXED, torch.float64, "scaled")
    else:
        _check(lib, orc, x, k, MIXED, torch.float64, "scaled", **variant)
    lib.close()


def test_large_level_sampled_rows():
    """Level 10 on the square (2.1 M unknowns): sampled rows against the
    oracle's rows assembled from the same node values (the oracle on a
    small patch around each sampled node equals the full operator's row)."""
    from paper_1908_08666_amd.twod import Mesh2D
    L = 10
    lib = Mesh2D(W.twod_mesh("square"), L, **EFORM)
    xy = lib.coords().T
    rng = np.random.default_rng(13)
    kf = lambda p: np.exp(0.5 * np.sin(7 * p[:, 0]) * np.cos(5 * p[:, 1]))      # noqa: E731
    xf = lambda p: np.column_stack([np.sin(13 * p[:, 0] + 3 * p[:, 1]), np.cos(11 * p[:, 1] - p[:, 0])])  # noqa: E731
    xt = torch.from_numpy(np.ascontiguousarray(xf(xy).T)).cuda()
    kt = torch.from_numpy(kf(xy)).cuda()
    y = lib.apply_scaled(xt, kt).cpu().numpy()
    flags = lib.flags()
    h = 1.0 / (1 << L)
    # oracle on a level-3 sub-square around each sampled node: same lattice
    # spacing, the node in its interior, every entry of its row present
    cand = np.nonzero(((flags & 1) == 0))[0]
    sample = rng.choice(cand, 300, replace=False)
    errs = []
    for s in sample:
        p = xy[s]
        lo = np.clip(np.round(p / h) - 4, 0, (1 << L) - 8) * h
        sub = W.twod_mesh("square") * (8 * h) + lo
        orc = T2.Mesh2D(sub, 3, dirichlet="none")
        A = T2.scaled_matrix(orc, kf(orc.xy), EFORM)
        i = int(np.argmin(np.linalg.norm(orc.xy - p, axis=1)))
        # rows of nodes on the sub-square's boundary are incomplete there
        if np.any(np.abs(orc.xy[i] - lo) < 1e-12) or np.any(np.abs(orc.xy[i] - lo - 8 * h) < 1e-12):
            continue
        # x at Dirichlet nodes of the full mesh is read as 0
        xs = xf(orc.xy)
        dmask = (orc.xy[:, 0] < 1e-12) | (orc.xy[:, 1] < 1e-12) | (orc.xy[:, 0] > 1 - 1e-12) | (orc.xy[:, 1] > 1 - 1e-12)
        xs[dmask] = 0.0
        ref = (A @ xs.ravel()).reshape(-1, 2)[i]
        errs.append(np.abs(y[:, s] - ref).max() / max(np.abs(ref).max(), 1e-300))
    errs = np.array(errs)
    print(f"  level {L}: {len(errs)} sampled rows, max rel err {errs.max():.2e}", flush=True)
    assert len(errs) > 200 and errs.max() < 1e-10
    lib.close()


def test_rejects_bad_arguments():
    from paper_1908_08666_amd import _lib as L
    from paper_1908_08666_amd.twod import Mesh2D
    with pytest.raises(L.HHGError):
        Mesh2D(W.twod_mesh("square"), 0, **EFORM)
    lib = Mesh2D(W.twod_mesh("square"), 3, **EFORM)
    x = torch.zeros(2, lib.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(L.HHGError):
        lib.apply_scaled(x, x[0].clone(), y=x)
    lib.close()
