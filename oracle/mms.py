"""Manufactured solution of the compressible Navier-Stokes equations
(ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

Sec. 7 (manufactured solution for the compressible Navier-Stokes equations):
on a periodic box the fields

    rho = rho0 + a sin(pi (sum_i x_i - c t)),   V_i = V0,
    p   = (gamma - 1) (rho^2 - rho |V|^2 / 2)

(the paper: rho0 = 2, a = 0.1, c = 0.6, V0 = 1 in every direction) solve
du/dt + sum_i dF^I_i/dx_i = sum_i dF^V_i/dx_i + S with the source

    S = du/dt + sum_i dF^I_i/dx_i - sum_i dF^V_i/dx_i

obtained by substituting the fields into the equations of Sec. 2.2.  This
module writes that definition out term by term from the derivatives of rho:
the time derivative of each conserved variable, the divergence of each
inviscid flux entry and of the viscous flux (the stress vanishes for a
constant velocity; the heat flux kappa dT/dx_i remains when it is switched
on).  The paper gives neither the period nor the source in closed form; the
fields have period 2 in every x_i, so any periodic box with sides a multiple
of 2 (the paper's [-1, 1]^d) carries them.

The error of the grid studies follows the paper's accuracy section (Sec.
7.3): the nodal solution is interpolated to a quadrature rule of degree
3p + 1, the squared error integrated over each element and summed.  The
paper does not say how n_p > dim P_p nodal values are interpolated; here it
is the least-squares fit of degree p weighted by the reference diagonal
norm h (exact for degree-p polynomials), evaluated at the points of a
collapsed Gauss-Legendre rule exact to degree 3p + 1 on the unit simplex.

Parity: pinned in tests/test_oracle_mms.py by fourth-order central
differences of physics.flux and physics.viscous_flux applied to the fields
(an independent route to the same source), by the vanishing source of a
constant state (a = 0), and by the total energy rho^2 that the paper's
pressure gives when |V|^2 = d; the quadrature norm by exact monomial
integrals on the simplex, exact reproduction of degree-p polynomials, a
constant offset integrating to its square times the box volume on curved
and affine grids, and the p + 1 decay of the interpolation error; the 3D vortex by the
Euler equations it satisfies (fourth-order differences of physics.flux).
"""
from __future__ import annotations

import numpy as np

PAPER = (2.0, 0.1, 0.6, 1.0)  # rho0, a, c, V0


def _rho_derivs(x, t, par):
    """rho and its derivatives: rho_t, rho_i (the same for every i), rho_ii."""
    rho0, a, c, _ = par
    xi = np.pi * (np.sum(x, axis=0) - c * t)
    rho = rho0 + a * np.sin(xi)
    rho_x = a * np.pi * np.cos(xi)
    rho_t = -c * rho_x
    rho_xx = -a * np.pi ** 2 * np.sin(xi)
    return rho, rho_t, rho_x, rho_xx


def state(x, t, gas, par=PAPER):
    """Conservative state U[d+2, ...] at points x[d, ...] and time t."""
    d = x.shape[0]
    V0 = par[3]
    rho, _, _, _ = _rho_derivs(x, t, par)
    q2 = d * V0 * V0
    p = (gas.gamma - 1.0) * (rho * rho - 0.5 * rho * q2)
    e = p / (gas.gamma - 1.0) + 0.5 * rho * q2
    return np.stack([rho] + [rho * V0] * d + [e], 0)


def source(x, t, gas, par=PAPER, viscous=True):
    """S[d+2, ...] = du/dt + div F^I - div F^V at points x[d, ...], time t.

    viscous=False drops the viscous flux (Euler equations with the same
    fields); with viscous=True the heat flux enters when gas.heat_flux."""
    d = x.shape[0]
    g = gas.gamma
    V0 = par[3]
    rho, rho_t, rho_x, rho_xx = _rho_derivs(x, t, par)
    q2 = d * V0 * V0
    # pressure and its derivatives (p = (g-1)(rho^2 - rho q2/2))
    p = (g - 1.0) * (rho * rho - 0.5 * rho * q2)
    dp_drho = (g - 1.0) * (2.0 * rho - 0.5 * q2)
    p_t, p_x = dp_drho * rho_t, dp_drho * rho_x
    p_xx = (g - 1.0) * 2.0 * rho_x * rho_x + dp_drho * rho_xx
    # total energy e = p/(g-1) + rho q2/2
    e_t = p_t / (g - 1.0) + 0.5 * q2 * rho_t
    e_x = p_x / (g - 1.0) + 0.5 * q2 * rho_x
    S = []
    # mass: d rho/dt + sum_i d(rho V_i)/dx_i
    S.append(rho_t + d * V0 * rho_x)
    # momentum j: d(rho V_j)/dt + sum_i d(rho V_i V_j)/dx_i + dp/dx_j
    for _ in range(d):
        S.append(V0 * rho_t + d * V0 * V0 * rho_x + p_x)
    # energy: de/dt + sum_i d((e + p) V_i)/dx_i - sum_i d(kappa dT/dx_i)/dx_i
    en = e_t + d * V0 * (e_x + p_x)
    if viscous and gas.heat_flux:
        R = gas.R
        # T = p / (rho R): second derivative along one x_i (quotient rule)
        T_xx = (p_xx / rho - 2.0 * p_x * rho_x / rho ** 2 - p * rho_xx / rho ** 2
                + 2.0 * p * rho_x ** 2 / rho ** 3) / R
        en = en - gas.kappa * d * T_xx
    S.append(en)
    return np.stack(S, 0)


def l2_error(u, x, t, H, gas, par=PAPER):
    """Per component sum_k (u_k - u*)^T H_k (u_k - u*) over the mesh, u[ne, n_c, n_p],
    x[ne, d, n_p] node coordinates, H[ne, n_p]."""
    ue = state(np.moveaxis(x, 1, 0), t, gas, par)       # [n_c, ne, n_p]
    err = u - np.moveaxis(ue, 0, 1)
    return np.einsum("en,ecn->c", H, err * err)


def vortex3d_state(x, t, gas):
    """The 3D isentropic vortex of the accuracy study (Sec. 7.3) at points
    x[3, ...], time t: with r^2 = x1^2 + (x2 - t)^2 and g = exp(1 - r^2),
      rho = (1 - 2/25 (gamma - 1) g)^(1/(gamma - 1)),
      V = (-2/5 (x2 - t) g^(1/2), 1 + 2/5 x1 g^(1/2), 0),
      e = rho^gamma / (gamma (gamma - 1)) + rho |V|^2 / 2  (p = rho^gamma / gamma).
    The printed exponent of V_1 is garbled; it is read as that of V_2 (the
    vortex centred on the x2 axis, advected along x2 at unit speed)."""
    g = gas.gamma
    y = x[1] - t
    ex = np.exp(1.0 - x[0] ** 2 - y ** 2)
    rho = (1.0 - 2.0 / 25.0 * (g - 1.0) * ex) ** (1.0 / (g - 1.0))
    V1 = -0.4 * y * np.sqrt(ex)
    V2 = 1.0 + 0.4 * x[0] * np.sqrt(ex)
    p = rho ** g / g
    e = p / (g - 1.0) + 0.5 * rho * (V1 * V1 + V2 * V2)
    return np.stack([rho, rho * V1, rho * V2, 0.0 * rho, e], 0)


def simplex_rule(dim, k):
    """Collapsed Gauss-Legendre rule on the unit simplex exact for total
    degree k: points [nq, dim], weights [nq] (summing to 1/dim!)."""
    q = (k + dim + 1) // 2          # 2q - 1 >= k + dim - 1
    x, w = np.polynomial.legendre.leggauss(q)
    t, wt = 0.5 * (x + 1.0), 0.5 * w
    pts, wts = [], []
    if dim == 2:
        for i in range(q):
            for j in range(q):
                pts.append((t[i] * (1.0 - t[j]), t[j]))
                wts.append(wt[i] * wt[j] * (1.0 - t[j]))
    else:
        for i in range(q):
            for j in range(q):
                for l in range(q):
                    pts.append((t[i] * (1.0 - t[j]) * (1.0 - t[l]), t[j] * (1.0 - t[l]), t[l]))
                    wts.append(wt[i] * wt[j] * wt[l] * (1.0 - t[j]) * (1.0 - t[l]) ** 2)
    return np.array(pts), np.array(wts)


def _monomials(xi, p):
    dim = xi.shape[1]
    cols = []
    if dim == 2:
        for a in range(p + 1):
            for b in range(p + 1 - a):
                cols.append(xi[:, 0] ** a * xi[:, 1] ** b)
    else:
        for a in range(p + 1):
            for b in range(p + 1 - a):
                for c in range(p + 1 - a - b):
                    cols.append(xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
    return np.stack(cols, 1)


def interp_matrix(nodes, h, p, xq):
    """[nq, n_p]: degree-p least-squares fit to nodal values, weighted by h,
    evaluated at the points xq (reference coordinates)."""
    V = _monomials(np.asarray(nodes), p)
    sw = np.sqrt(np.asarray(h))[:, None]
    P = np.linalg.lstsq(sw * V, np.diag(sw[:, 0]), rcond=None)[0]   # [N, n_p]
    return _monomials(np.asarray(xq), p) @ P


def l2_error_quadrature(u, mesh, exact):
    """Per component sum_k integral over element k of (I u_k - u*)^2 with the
    degree-(3p+1) rule; u[ne, n_c, n_p], mesh an OracleMesh, exact(x[d, n]) ->
    [n_c, n]."""
    from .geometry import _p2_basis, _p2_basis3
    xq, wq = simplex_rule(mesh.dim, 3 * mesh.p + 1)
    I = interp_matrix(mesh.ops["nodes"], mesh.ops["h"], mesh.p, xq)
    if mesh.p_geom == 2:
        N, dN = _p2_basis(xq) if mesh.dim == 2 else _p2_basis3(xq)
    out = np.zeros(mesh.n_c)
    for e in range(mesh.ne):
        if mesh.p_geom == 2:
            g = np.asarray(mesh.geom_nodes[e], dtype=np.float64)        # [6, 2] or [10, 3]
            x = g.T @ N                                              # [d, nq]
            F = np.einsum("ai,lan->nil", g, dN)                     # dx_i/dxi_l per point
            J = np.linalg.det(F)
        else:
            v = mesh.verts[mesh.elem[e]]                             # [d+1, d]
            F = np.stack([v[l + 1] - v[0] for l in range(mesh.dim)], 1)
            x = v[0][:, None] + F @ xq.T
            J = np.full(len(wq), np.linalg.det(F))
        err = u[e] @ I.T - exact(x)                                  # [n_c, nq]
        out += np.sum(wq * J * err * err, axis=1)
    return out
