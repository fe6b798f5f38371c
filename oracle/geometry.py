"""Physical SBP operators on mapped elements and facet coupling data
(ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

Sec. 2.1 defines the physical operators only through Def. 1 and Assumption 1
and refers to the literature for curved elements.  The reading taken here:
  * the element map is affine (p_geom = 1) or quadratic through the vertices
    and edge midpoints (p_geom = 2; Assumption 1 allows it for p >= 1 in 2D
    and p >= 2 in 3D);
  * metric terms Lambda_{il} = J d(xi_l)/d(x_i) (cofactors of dx/dxi) at the
    SBP nodes, H_k = diag(J) H_ref;
  * Q_{x_i,k} = 1/2 sum_l (Lambda_il Q_xi_l + Q_xi_l Lambda_il) with the
    diagonal matrices Lambda_il, hence E_{x_i,k} = sum_l Lambda_il E_xi_l and
    the SBP property of Def. 1 holds;
  * the facet weight-times-normal B n_i at a facet node is the diagonal entry
    of E_{x_i,k} there (decomposition of E in Sec. 2.1).

Facet matching: facets are identified by their vertex centroids modulo the
periodic box; facet nodes are paired by coordinates modulo the box.

Parity: pinned by tests/test_oracle_geometry.py (SBP property and exactness
of the physical operators on affine elements, Q_x 1 = 0 on curved elements,
B n from the two sides equal and opposite, matched node coordinates).
"""
from __future__ import annotations

import numpy as np

from .operators import reference_operator


def _p2_basis(xi):
    """Quadratic Lagrange basis on the reference triangle, node order
    v0, v1, v2, mid(v0,v1), mid(v1,v2), mid(v2,v0); returns (N[6,n], dN[2,6,n])."""
    x, y = xi[:, 0], xi[:, 1]
    l0, l1, l2 = 1.0 - x - y, x, y
    dl = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # d lambda_a / d xi_l
    lam = [l0, l1, l2]
    N = np.array([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                  4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0])
    dN = np.zeros((2, 6, len(x)))
    for l in range(2):
        for a in range(3):
            dN[l, a] = (4 * lam[a] - 1) * dl[a, l]
        for q, (a, b) in enumerate([(0, 1), (1, 2), (2, 0)]):
            dN[l, 3 + q] = 4 * (dl[a, l] * lam[b] + lam[a] * dl[b, l])
    return N, dN


P2_TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def _p2_basis3(xi):
    """Quadratic Lagrange basis on the reference tetrahedron, node order
    v0..v3 then the edge midpoints in P2_TET_EDGES order; returns
    (N[10,n], dN[3,10,n])."""
    n = xi.shape[0]
    lam = [1.0 - xi[:, 0] - xi[:, 1] - xi[:, 2], xi[:, 0], xi[:, 1], xi[:, 2]]
    dl = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    N = np.zeros((10, n))
    dN = np.zeros((3, 10, n))
    for a in range(4):
        N[a] = lam[a] * (2 * lam[a] - 1)
        for l in range(3):
            dN[l, a] = (4 * lam[a] - 1) * dl[a, l]
    for q, (a, b) in enumerate(P2_TET_EDGES):
        N[4 + q] = 4 * lam[a] * lam[b]
        for l in range(3):
            dN[l, 4 + q] = 4 * (dl[a, l] * lam[b] + lam[a] * dl[b, l])
    return N, dN


def _wrap_key(c, period, res=1 << 22):
    return tuple(int(round(c[i] / period[i] * res)) % res for i in range(len(c)))


class OracleMesh:
    """Mesh of one degree p built from a mesh description (see
    paper_2305_07181_amd.workloads).  Geometry is computed per element on
    demand; connectivity for all facets at construction."""

    def __init__(self, desc: dict, p: int):
        self.dim = int(desc["dim"])
        self.p = int(p)
        self.ops = reference_operator(self.dim, self.p)
        self.verts = np.asarray(desc["vert_xyz"], dtype=np.float64)
        self.elem = np.asarray(desc["elem_vert"], dtype=np.int64)
        self.period = np.asarray(desc["period"], dtype=np.float64)
        self.p_geom = int(desc.get("p_geom", 1))
        self.geom_nodes = desc.get("geom_nodes")
        self.ne = len(self.elem)
        self.n_p = self.ops["n_p"]
        self.n_c = self.dim + 2
        self.n_fac = self.dim + 1
        self._geo = {}
        self._match_facets()
        self._perm = {}

    # ---------------- connectivity -----------------
    def _facet_vertex_ids(self, f):
        return [i for i in range(self.dim + 1) if i != f]

    def _match_facets(self):
        table = {}
        for e in range(self.ne):
            for f in range(self.n_fac):
                vs = self.verts[self.elem[e, self._facet_vertex_ids(f)]]
                key = _wrap_key(vs.mean(axis=0), self.period)
                table.setdefault(key, []).append((e, f))
        self.nbr = -np.ones((self.ne, self.n_fac, 2), dtype=np.int64)
        for key, lst in table.items():
            if len(lst) != 2:
                raise ValueError(f"facet shared by {len(lst)} elements")
            (e1, f1), (e2, f2) = lst
            self.nbr[e1, f1] = (e2, f2)
            self.nbr[e2, f2] = (e1, f1)

    def neighbor(self, e, f):
        v, g = self.nbr[e, f]
        return int(v), int(g)

    def facet_perm(self, e, f):
        """perm[j] = index (within the neighbor facet's node list) of the node
        matching node j of facet f of element e."""
        key = (e, f)
        if key in self._perm:
            return self._perm[key]
        v, g = self.neighbor(e, f)
        xe = self.geometry(e)["x"][self.ops["facet_nodes"][f]]
        xv = self.geometry(v)["x"][self.ops["facet_nodes"][g]]
        h = self.geometry(e)["h_min"]
        perm = []
        for j in range(len(xe)):
            dd = xv - xe[j]
            dd = dd - self.period * np.round(dd / self.period)
            dist = np.linalg.norm(dd, axis=1)
            q = int(np.argmin(dist))
            if dist[q] > 1e-8 * max(h, 1.0):
                raise ValueError("facet nodes do not match")
            perm.append(q)
        perm = np.array(perm)
        self._perm[key] = perm
        return perm

    # ---------------- geometry -----------------
    def geometry(self, e):
        if e in self._geo:
            return self._geo[e]
        ops = self.ops
        dim = self.dim
        xi = ops["nodes"]
        n_p = len(xi)
        if self.p_geom == 1:
            v = self.verts[self.elem[e]]
            F = np.stack([v[l + 1] - v[0] for l in range(dim)], 1)  # F[i,l] = dx_i/dxi_l
            x = v[0][None, :] + xi @ F.T
            Fn = np.broadcast_to(F, (n_p, dim, dim)).copy()
        elif self.p_geom == 2:
            g = np.asarray(self.geom_nodes[e], dtype=np.float64)  # [6,2] or [10,3]
            N, dN = _p2_basis(xi) if dim == 2 else _p2_basis3(xi)
            x = N.T @ g
            Fn = np.zeros((n_p, dim, dim))
            for l in range(dim):
                Fn[:, :, l] = dN[l].T @ g
        else:
            raise ValueError("unsupported geometry")
        J = np.linalg.det(Fn)
        # Lambda[m, i, l] = J dxi_l/dx_i = J (F^{-1})[l, i]
        Finv = np.linalg.inv(Fn)
        Lam = J[:, None, None] * np.transpose(Finv, (0, 2, 1))
        H = J * ops["h"]
        Qx = np.zeros((dim, n_p, n_p))
        Ex = np.zeros((dim, n_p))
        for i in range(dim):
            for l in range(dim):
                lam = Lam[:, i, l]
                Qx[i] += 0.5 * (lam[:, None] * ops["Q"][l] + ops["Q"][l] * lam[None, :])
                Ex[i] += lam * ops["E"][l]
        Dx = Qx / H[None, :, None]
        Bn = np.zeros((self.n_fac, ops["n_f"], dim))
        for f in range(self.n_fac):
            for j, m in enumerate(ops["facet_nodes"][f]):
                Bn[f, j] = Ex[:, m]
        dif = x[:, None, :] - x[None, :, :]
        dist = np.linalg.norm(dif, axis=2)
        h_min = dist[np.triu_indices(n_p, 1)].min()
        geo = dict(x=x, J=J, Lam=Lam, H=H, Qx=Qx, Ex=Ex, Dx=Dx, Bn=Bn, h_min=h_min)
        self._geo[e] = geo
        return geo

    def node_coords(self, elements=None):
        """SBP node coordinates [ne, dim, n_p] (component-first per element),
        from the element maps only (no operators), vectorised over elements."""
        els = np.arange(self.ne) if elements is None else np.asarray(list(elements))
        xi = self.ops["nodes"]
        if self.p_geom == 1:
            v = self.verts[self.elem[els]]                      # [n, dim+1, dim]
            F = np.stack([v[:, l + 1] - v[:, 0] for l in range(self.dim)], 2)  # [n, i, l]
            x = v[:, 0][:, None, :] + np.einsum("jl,nil->nji", xi, F)
        else:
            N, _ = _p2_basis(xi) if self.dim == 2 else _p2_basis3(xi)
            g = np.asarray(self.geom_nodes, dtype=np.float64)[els]   # [n,6,2] or [n,10,3]
            x = np.einsum("aj,nai->nji", N, g)
        return np.ascontiguousarray(np.transpose(x, (0, 2, 1)))

    def H_all(self):
        return np.stack([self.geometry(e)["H"] for e in range(self.ne)], 0)
