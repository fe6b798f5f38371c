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

Parity: pinned in tests/test_oracle_mms.py by fourth-order central
differences of physics.flux and physics.viscous_flux applied to the fields
(an independent route to the same source), by the vanishing source of a
constant state (a = 0), and by the total energy rho^2 that the paper's
pressure gives when |V|^2 = d.
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
