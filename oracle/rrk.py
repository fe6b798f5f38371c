"""Relaxation RK4 (ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

Sec. 6.1 (eqs. rrk4 gamma_n and rrk_update): classical four-stage RK4 stages
r_i, direction d = dt sum_i b_i r_i, entropy production estimate
e = dt sum_i b_i w_i^T H r_i, and gamma_n solving
    1^T H s(u_n + gamma d) - 1^T H s(u_n) - gamma e = 0
by bisection; u_{n+1} = u_n + gamma_n d.

Readings: classical RK4 tableau; the equality is solved also with
dissipation; bracket [0.5, 1.5]; bisection stops when the midpoint equals an
endpoint; the entropy difference is summed node by node; t_{n+1} = t_n +
gamma_n dt.

Parity: pinned by tests/test_oracle_rrk.py (the fully discrete entropy
equality holds to roundoff, gamma -> 1 as dt -> 0, fourth-order accuracy of
the underlying RK4 on a linear ODE).
"""
from __future__ import annotations

import numpy as np

from . import physics as ph

B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
C_STAGE = (0.0, 0.5, 0.5, 1.0)


def rk4_direction(scheme, u, dt, source=None, t=0.0):
    """Return (d, e) for one RK4 step from u.  source(t) -> [ne, n_c, n_p]
    (a manufactured-solution source, Sec. 7) is added to every stage
    residual at the stage time t + c_i dt when given."""
    gas = scheme.gas
    H = scheme.mesh.H_all()
    d = np.zeros_like(u)
    e = 0.0
    y = u
    for i in range(4):
        if i > 0:
            y = u + C_STAGE[i] * dt * r
        r = scheme(y)
        if source is not None:
            r = r + source(t + C_STAGE[i] * dt)
        w = np.stack([ph.entropy_vars(y[k], gas) for k in range(len(y))], 0)
        e = e + dt * B[i] * np.sum(H[:, None, :] * w * r)
        d = d + dt * B[i] * r
    return d, e


def entropy_gap(scheme, u, d, e, gamma, H=None):
    """r(gamma) = sum_nodes H [s(u + gamma d) - s(u)] - gamma e."""
    gas = scheme.gas
    H = scheme.mesh.H_all() if H is None else H
    s1 = ph.entropy(np.moveaxis(u + gamma * d, 1, 0), gas)   # [ne, n_p]
    s0 = ph.entropy(np.moveaxis(u, 1, 0), gas)
    return float(np.sum(H * (s1 - s0)) - gamma * e)


def solve_gamma(scheme, u, d, e, lo=0.5, hi=1.5, max_iter=200):
    H = scheme.mesh.H_all()
    flo = entropy_gap(scheme, u, d, e, lo, H)
    fhi = entropy_gap(scheme, u, d, e, hi, H)
    if not (flo < 0.0 < fhi):
        raise RuntimeError(f"relaxation root not bracketed: r({lo})={flo}, r({hi})={fhi}")
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        fm = entropy_gap(scheme, u, d, e, mid, H)
        if fm == 0.0:
            lo = hi = mid
            break
        if fm < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def rrk4_step(scheme, u, dt, source=None, t=0.0):
    """One relaxation RK4 step; returns (u_new, gamma, d, e)."""
    d, e = rk4_direction(scheme, u, dt, source, t)
    gamma = solve_gamma(scheme, u, d, e)
    return u + gamma * d, gamma, d, e
