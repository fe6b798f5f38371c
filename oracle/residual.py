"""Semi-discrete residuals du/dt = r(u) (ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

Per element k, with c_b = 1/(beta+1), physical operators from geometry.py,
the entropy-split scheme in its efficient (weak) form (Sec. 6.2, eq. weak form
split) is

  r_k = H^-1 sum_i [c_b Q_xi + Q_xi^T] f^(i) - c_b sum_i A~_i D_xi w
        - 1/2 H^-1 sum_{gamma} sum_i [E^{kv}_xi o F_i(u_k, u_v)] 1        (EC SAT)
        - 1/2 H^-1 R^T B X|Lambda|S X^T (w_k - w_v)          (dissipation, Sec. 4.5)
        + sum_i sum_j D_xi K~_ij D_xj w + SAT^V                     (Sec. 5)

The coupling term reduces, for diagonal-E operators and the factor 2 inside
F_i (eq. F 2-point), to -(B n . F*(u_k, u_v)) / H at every facet node.  The
Hadamard form (Sec. 6.2, eq. weak form 2pt) replaces the first line by
-H^-1 sum_i [S_xi o F_i(u_k, u_k)] 1.  The hybrid scheme (Sec. 4.4, Thm.
switching hybrid) takes, element by element, either of the two volume terms
with the same SATs (form 'hybrid', per-element flags 0 = split, 1 =
Hadamard).  The strong form (Sec. 4, eqs. discrete entropy split and sats
inv) is provided for the strong = weak cross-check.
Baumann-Oden viscous SATs (Sec. 5.1, eq. bo sats): T1 = 0, T2 = T3 = B/2.

Readings: the stray w_k^T in the printed Hadamard weak form is
dropped; the coupling sums run over the facets of element k.

Parity: pinned by tests/test_oracle_residual.py: free-stream preservation,
entropy conservation sum w^T H r = 0 (Thm. entropy conservation) for the split
and Hadamard forms, sum w^T H r <= 0 with dissipation and with heat-flux-free
viscous terms, the per-element volume identity w^T H r_vol = sum_i 1^T E_xi
psi^(i) (Lemma entropy conv volume), strong = weak, vanishing SATs for
continuous states (Lemma sats vanish), Hadamard local conservation, the
hybrid scheme's entropy conservation with random flags (also switched between
RRK steps) and local conservation on its Hadamard elements, and design-order
truncation error on smooth states (Thm. high-order).  The kinetic energy:
tests/test_oracle_tgv.py (a uniform flow gives rho |V|^2 / 2 times the
volume; the Taylor-Green initial field gives E_k -> 1/8, its closed form,
under refinement).  The time step (Sec. 7.1): tests/test_oracle_timestep.py
(closed-form h_min of the Gauss-Legendre edge nodes on uniform grids, the
ratio under refinement, the fastest and the smallest element deciding).
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from .geometry import OracleMesh


class OracleScheme:
    """Residual evaluator.  form: 'split' (entropy split), 'hadamard', or
    'hybrid' with element_form[e] = 0 (split) or 1 (Hadamard) per element;
    element_form may be reassigned between calls (switching between steps)."""

    def __init__(self, mesh: OracleMesh, gas: ph.Gas, form="split",
                 dissipation=False, viscous=False, element_form=None):
        if form not in ("split", "hadamard", "hybrid"):
            raise ValueError(form)
        if (form == "hybrid") != (element_form is not None):
            raise ValueError("element_form is given exactly for the hybrid form")
        self.mesh = mesh
        self.gas = gas
        self.form = form
        self.element_form = None if element_form is None else np.asarray(element_form, dtype=int)
        self.dissipation = bool(dissipation)
        self.viscous = bool(viscous)
        self.cb = 1.0 / (gas.beta + 1.0)

    # ------------------------------------------------------------------
    def volume_split(self, U, geo):
        """H^-1 sum_i [c_b Q_xi + Q_xi^T] f^(i) - c_b sum_i A~_i D_xi w."""
        d = self.mesh.dim
        gas = self.gas
        w = ph.entropy_vars(U, gas)
        acc = 0.0
        for i in range(d):
            f = ph.flux(U, i, gas)
            M = self.cb * geo["Qx"][i] + geo["Qx"][i].T
            acc = acc + M @ f.T                     # [n_p, n_c]
        r = (acc / geo["H"][:, None]).T
        for i in range(d):
            Dw = geo["Dx"][i] @ w.T                  # [n_p, n_c]
            At = ph.symmetrized_jacobian(U, i, gas)  # [n_c, n_c, n_p]
            r = r - self.cb * np.einsum("abm,mb->am", At, Dw)
        return r

    def volume_split_strong(self, U, geo):
        """-beta/(beta+1) sum_i D_xi f - c_b sum_i A~_i D_xi w + H^-1 sum_i E_xi f."""
        d = self.mesh.dim
        gas = self.gas
        w = ph.entropy_vars(U, gas)
        beta = gas.beta
        r = 0.0
        for i in range(d):
            f = ph.flux(U, i, gas)
            r = r - beta / (beta + 1.0) * (geo["Dx"][i] @ f.T).T
            r = r + geo["Ex"][i][None, :] * f / geo["H"][None, :]
            Dw = geo["Dx"][i] @ w.T
            At = ph.symmetrized_jacobian(U, i, gas)
            r = r - self.cb * np.einsum("abm,mb->am", At, Dw)
        return r

    def volume_hadamard(self, U, geo):
        """-H^-1 sum_i [S_xi o F_i(u_k,u_k)] 1, F_i carrying the factor 2."""
        d = self.mesh.dim
        Fs = ph.sy_flux(U[:, :, None], U[:, None, :], self.gas)  # [d,n_c,m,n]
        r = 0.0
        for i in range(d):
            Sx = geo["Qx"][i] - 0.5 * np.diag(geo["Ex"][i])
            r = r - 2.0 * np.einsum("mn,amn->am", Sx, Fs[i])
        return r / geo["H"][None, :]

    # ------------------------------------------------------------------
    def _viscous_data(self, u, e, cache):
        """grad W (D_x w), A0, K~ products and F^V at all nodes of element e."""
        if e in cache:
            return cache[e]
        mesh, gas = self.mesh, self.gas
        d = mesh.dim
        geo = mesh.geometry(e)
        U = u[e]
        w = ph.entropy_vars(U, gas)
        gw = np.stack([(geo["Dx"][j] @ w.T).T for j in range(d)], 0)   # [d, n_c, n_p]
        A0 = ph.dU_dW(U, gas)                                          # [n_c, n_c, n_p]
        gU = np.einsum("abm,jbm->jam", A0, gw)
        FV = ph.viscous_flux(U, gU, gas)                                # [d(i), n_c, n_p]
        out = dict(w=w, FV=FV, A0=A0)
        cache[e] = out
        return out

    def _Ktilde(self, U, A0):
        """K~[i][j] : [n_c, n_c, n_p] with F^V(i) = sum_j K~_ij dW/dx_j,
        assembled column by column from unit entropy-variable gradients."""
        d = self.mesh.dim
        nc = d + 2
        n_p = U.shape[1]
        K = np.zeros((d, d, nc, nc, n_p), dtype=np.result_type(U, 1.0))
        for j in range(d):
            for c in range(nc):
                G = np.zeros((d, nc, n_p), dtype=K.dtype)
                G[j] = A0[:, c, :]
                FV = ph.viscous_flux(U, G, self.gas)
                for i in range(d):
                    K[i, j, :, c, :] = FV[i]
        return K

    # ------------------------------------------------------------------
    def element(self, u, e, vcache=None, strong=False):
        mesh, gas = self.mesh, self.gas
        ops = mesh.ops
        geo = mesh.geometry(e)
        U = u[e]
        split = self.form == "split" or (self.form == "hybrid" and self.element_form[e] == 0)
        if split:
            r = self.volume_split_strong(U, geo) if strong else self.volume_split(U, geo)
        else:
            if strong:
                raise ValueError("strong form only for the split scheme")
            r = self.volume_hadamard(U, geo)
        H = geo["H"]
        w = ph.entropy_vars(U, gas) if (self.dissipation or self.viscous) else None
        for f in range(mesh.n_fac):
            v, g = mesh.neighbor(e, f)
            perm = mesh.facet_perm(e, f)
            mk = ops["facet_nodes"][f]
            mv = ops["facet_nodes"][g][perm]
            Uk = U[:, mk]
            Uv = u[v][:, mv]
            Bn = geo["Bn"][f]                       # [n_f, d]
            Fs = ph.sy_flux(Uk, Uv, gas)            # [d, n_c, n_f]
            nF = np.einsum("jd,dcj->cj", Bn, Fs)
            r[:, mk] = r[:, mk] - nF / H[None, mk]
            if self.dissipation:
                wv = ph.entropy_vars(Uv, gas)
                for j in range(len(mk)):
                    B = np.linalg.norm(Bn[j])
                    n = Bn[j] / B
                    Md = ph.dissipation_matrix(Uk[:, j], Uv[:, j], n, gas)
                    r[:, mk[j]] = r[:, mk[j]] - 0.5 * B / H[mk[j]] * (Md @ (w[:, mk[j]] - wv[:, j]))
        if self.viscous:
            r = r + self._viscous_element(u, e, vcache if vcache is not None else {})
        return r

    def _viscous_element(self, u, e, cache):
        mesh, gas = self.mesh, self.gas
        ops = mesh.ops
        d = mesh.dim
        geo = mesh.geometry(e)
        H = geo["H"]
        dk = self._viscous_data(u, e, cache)
        FV = dk["FV"]
        rv = 0.0
        for i in range(d):
            rv = rv + (geo["Dx"][i] @ FV[i].T).T
        K = self._Ktilde(u[e], dk["A0"])
        y = np.zeros((d, self.mesh.n_c, self.mesh.n_p), dtype=rv.dtype)
        for f in range(mesh.n_fac):
            v, g = mesh.neighbor(e, f)
            perm = mesh.facet_perm(e, f)
            mk = ops["facet_nodes"][f]
            mv = ops["facet_nodes"][g][perm]
            dv = self._viscous_data(u, v, cache)
            Bn = geo["Bn"][f]                       # [n_f, d]
            jumpF = np.einsum("jd,dcj->cj", Bn, FV[:, :, mk] - dv["FV"][:, :, mv])
            rv[:, mk] = rv[:, mk] - 0.5 * jumpF / H[None, mk]
            dw = dk["w"][:, mk] - dv["w"][:, mv]   # [n_c, n_f]
            for jj in range(d):
                for i in range(d):
                    # K~_ij^T (B n_i dw)
                    y[jj][:, mk] += np.einsum("bam,bm->am", K[i, jj][:, :, mk], Bn[:, i][None, :] * dw)
        for jj in range(d):
            rv = rv - 0.5 * (geo["Dx"][jj].T @ y[jj].T).T / H[None, :]
        return rv

    def __call__(self, u, elements=None, strong=False):
        els = range(self.mesh.ne) if elements is None else elements
        vcache = {}
        out = np.stack([self.element(u, e, vcache, strong=strong) for e in els], 0)
        return out

    # ------------------------------------------------------------------
    def entropy_rate(self, u, r):
        """sum_k w_k^T H_k r_k."""
        tot = 0.0
        for e in range(self.mesh.ne):
            w = ph.entropy_vars(u[e], self.gas)
            tot = tot + np.sum(self.mesh.geometry(e)["H"][None, :] * w * r[e])
        return tot

    def total_entropy(self, u):
        """s = 1^T H_g s(u)."""
        return sum(np.sum(self.mesh.geometry(e)["H"] * ph.entropy(u[e], self.gas))
                   for e in range(self.mesh.ne))

    def kinetic_energy(self, u):
        """1^T H_g (rho |V|^2 / 2): the integral whose scaled form
        E_k = (1 / (rho_0 |Omega|)) int rho V.V / 2 the viscous Taylor-Green
        study reports (Sec. 7.5)."""
        tot = 0.0
        for e in range(self.mesh.ne):
            rho, V, _ = ph.primitive(u[e], self.gas)
            tot = tot + np.sum(self.mesh.geometry(e)["H"] * 0.5 * rho * np.sum(V * V, axis=0))
        return tot

    def timestep(self, u, cfl):
        """dt = CFL min_k h_min,k / |lambda|_max,k (Sec. 7.1)."""
        best = np.inf
        for e in range(self.mesh.ne):
            rho, V, p = ph.primitive(u[e], self.gas)
            lam = np.max(np.sqrt(np.sum(V * V, axis=0)) + np.sqrt(self.gas.gamma * p / rho))
            best = min(best, cfl * self.mesh.geometry(e)["h_min"] / lam)
        return best
