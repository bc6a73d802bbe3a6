"""GPU nodal strain rate + Carreau viscosity against the oracle (Sec. 3)."""
import numpy as np
import pytest

import workloads as W
from oracle import strain as ST
from oracle.mesh import MacroMesh
from tests.helpers import slot_to_node, scatter

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAW = dict(eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25)


@pytest.mark.parametrize("name,verts,L,scale", [("cube24", W.cube24(), 3, 30.0),
                                                ("kuhn6", W.kuhn6(), 3, 5.0),
                                                ("unit", W.unit_tet(), 4, 100.0)])
def test_viscosity_matches_oracle(name, verts, L, scale):
    from paper_1908_08666_amd import Mesh
    lib = Mesh(verts, L, mu1=1.0)
    orc = MacroMesh(verts, L)
    s2n = slot_to_node(lib, orc)
    u = W.velocity_field(orc.xyz, W.rng_for(3, 4), scale)
    ut = torch.from_numpy(scatter(u, s2n)).cuda()
    k = lib.nodal_viscosity(ut, **LAW)
    torch.cuda.synchronize()
    kg = k.cpu().numpy()
    ref = ST.nodal_viscosity(orc, u, **LAW)
    # consistent over copies and equal to the oracle
    err = np.abs(kg - ref[s2n]) / ref[s2n]
    print(f"  {name}: max rel err {err.max():.2e}, viscosity range {ref.min():.3e}..{ref.max():.3e}")
    assert err.max() < 1e-12
    assert ref.max() / ref.min() > 2.0          # the field exercises the law


def test_viscosity_rejects_bad_law():
    from paper_1908_08666_amd import Mesh, _lib as L
    lib = Mesh(W.unit_tet(), 3, mu1=1.0)
    u = torch.zeros(3, lib.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(L.HHGError):
        lib.nodal_viscosity(u, eta0=1.0, eta_inf=0.0)
