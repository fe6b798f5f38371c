"""Dense residual Jacobians by complex step (ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

J[:, q] = Im r(u + i h e_q) / h with h = 1e-30 is exact to rounding for the
complex-analytic residual of residual.py (|.| is taken as sign(Re z) z and
branch choices use real parts).  The vector-Jacobian product is J^T lambda.
The paper has no adjoint; the checks are two exact consequences of its
theorems (tests/test_oracle_jacobian.py):
  * entropy conservation (Thm. entropy conservation) holds for every state,
    so differentiating sum w^T H r = 0 gives J^T (H w) = -(dW/dU) H r;
  * the Hadamard form is conservative for every state (Thm. switching hybrid),
    so 1^T H J = 0 per component.
"""
from __future__ import annotations

import numpy as np


def dense_jacobian(scheme, u, h=1e-30):
    """J with rows/columns ordered like u.ravel()."""
    n = u.size
    J = np.zeros((n, n))
    base = u.astype(complex)
    flat = base.reshape(-1)
    for q in range(n):
        flat[q] += 1j * h
        J[:, q] = np.imag(scheme(base)).reshape(-1) / h
        flat[q] -= 1j * h
    return J


def vjp(scheme, u, lam, J=None):
    """(dr/du)^T lambda."""
    J = dense_jacobian(scheme, u) if J is None else J
    return (J.T @ lam.reshape(-1)).reshape(u.shape)


def vjp_elements(scheme, u, lam, elements, h=1e-30):
    """(dr/du)^T lambda restricted to the given elements: for every value of
    such an element, one complex-step column evaluated on the element and its
    facet neighbours only (the only residuals that depend on it)."""
    mesh = scheme.mesh
    out = {}
    base = u.astype(complex)
    for e in elements:
        near = [e] + [mesh.neighbor(e, f)[0] for f in range(mesh.n_fac)]
        near = sorted(set(near))
        g = np.zeros(u.shape[1:])
        for c in range(u.shape[1]):
            for j in range(u.shape[2]):
                base[e, c, j] += 1j * h
                r = scheme(base, elements=near)
                g[c, j] = np.sum(lam[near] * np.imag(r)) / h
                base[e, c, j] -= 1j * h
        out[e] = g
    return out
