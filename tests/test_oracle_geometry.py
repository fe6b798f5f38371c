"""Pins for the oracle's physical operators and facet coupling (Sec. 2.1,
Def. 1, Assumption 1)."""
import numpy as np
import pytest

from oracle.geometry import OracleMesh
from paper_2305_07181_amd import workloads as wl


def _monos(deg, dim):
    if dim == 2:
        return [(a, b) for a in range(deg + 1) for b in range(deg + 1 - a)]
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a) for c in range(deg + 1 - a - b)]


MESHES = [("tri-affine", lambda: wl.periodic_tri_mesh(3, 2, 2.0, 1.5), (1, 2, 3, 4)),
          ("tri-curved", lambda: wl.vortex2d_mesh(3, warp=0.05), (1, 2, 3, 4)),
          ("tet-affine", lambda: wl.periodic_tet_mesh(2, 1.3), (1, 2, 3)),
          # quadratic maps need p >= 2 in 3D (Assumption 1: p_geom <= floor(p/2) + 1)
          ("tet-curved", lambda: wl.curved_tet_mesh(2, 1.3, 0.03), (2, 3))]


@pytest.mark.parametrize("name,make,ps", MESHES, ids=[m[0] for m in MESHES])
def test_physical_operators(name, make, ps):
    desc = make()
    for p in ps:
        m = OracleMesh(desc, p)
        for e in range(0, m.ne, max(1, m.ne // 5)):
            geo = m.geometry(e)
            x = geo["x"]
            assert (geo["J"] > 0).all()
            for i in range(m.dim):
                Q, E = geo["Qx"][i], geo["Ex"][i]
                assert np.abs(Q + Q.T - np.diag(E)).max() < 1e-13 * np.abs(Q).max()
                # discrete metric identity: free-stream preservation Q_x 1 = 0
                assert np.abs(Q @ np.ones(m.n_p)).max() < 1e-13 * np.abs(Q).max()
                if desc["p_geom"] == 1:
                    for mono in _monos(p, m.dim):
                        f = np.prod([x[:, k] ** mono[k] for k in range(m.dim)], 0)
                        if mono[i] == 0:
                            df = 0 * f
                        else:
                            mm = list(mono)
                            mm[i] -= 1
                            df = mono[i] * np.prod([x[:, k] ** mm[k] for k in range(m.dim)], 0)
                        scale = np.abs(geo["Dx"][i]).max() * (1 + np.abs(f).max())
                        assert np.abs(geo["Dx"][i] @ f - df).max() < 1e-12 * scale
            # H integrates the element measure
            if desc["p_geom"] == 1:
                v = m.verts[m.elem[e]]
                vol = abs(np.linalg.det(np.stack([v[k + 1] - v[0] for k in range(m.dim)], 1))) / (2 if m.dim == 2 else 6)
                assert abs(geo["H"].sum() - vol) < 1e-13 * vol


@pytest.mark.parametrize("name,make,ps", MESHES, ids=[m[0] for m in MESHES])
def test_facet_coupling(name, make, ps):
    """Matched facet nodes coincide (mod the period) and B n from the two
    sides is equal and opposite (E^{kv} = -(E^{vk})^T, Sec. 2.1)."""
    desc = make()
    total = 0.0
    for p in ps:
        m = OracleMesh(desc, p)
        fn = m.ops["facet_nodes"]
        area = 0.0
        for e in range(m.ne):
            for f in range(m.n_fac):
                v, g = m.neighbor(e, f)
                perm = m.facet_perm(e, f)
                ge, gv = m.geometry(e), m.geometry(v)
                d = ge["x"][fn[f]] - gv["x"][fn[g][perm]]
                d = d - m.period * np.round(d / m.period)
                assert np.abs(d).max() < 1e-12
                assert np.abs(ge["Bn"][f] + gv["Bn"][g][perm]).max() < 1e-13
                # reverse permutation is consistent
                back = m.facet_perm(v, g)
                assert (back[perm] == np.arange(len(perm))).all()
                area += np.linalg.norm(ge["Bn"][f], axis=1).sum()
        total = area
    assert total > 0
