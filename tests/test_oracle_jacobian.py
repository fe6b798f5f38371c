"""Pins for the oracle's complex-step Jacobian and VJP."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.geometry import OracleMesh
from oracle.jacobian import dense_jacobian
from oracle.residual import OracleScheme
from paper_2305_07181_amd import workloads as wl


def _setup(dim, p, form="split", diss=False):
    desc = wl.periodic_tri_mesh(2, 2, 1.0)
    m = OracleMesh(desc, p)
    x = m.node_coords()
    rho, V, pr = wl.random_smooth_state(np.moveaxis(x, 1, 0), seed=1, L=1.0)
    u = np.moveaxis(wl.conservative(rho, V, pr), 0, 1)
    u = u * (1 + 0.01 * np.random.default_rng(2).standard_normal(u.shape))
    return m, OracleScheme(m, ph.Gas(), form=form, dissipation=diss), u


@pytest.mark.parametrize("p", [1, 2])
def test_entropy_conservation_adjoint_identity(p):
    """J^T (H w) = -(dW/dU) H r for the entropy-conservative split scheme."""
    m, s, u = _setup(2, p)
    J = dense_jacobian(s, u)
    r = s(u)
    H = m.H_all()
    w = np.stack([ph.entropy_vars(u[e], s.gas) for e in range(m.ne)], 0)
    lhs = (J.T @ (H[:, None, :] * w).reshape(-1)).reshape(u.shape)
    rhs = np.zeros_like(u)
    for e in range(m.ne):
        Hs = ph.dU_dW(u[e], s.gas)     # dU/dW; dW/dU is its inverse
        Hw = np.linalg.inv(np.moveaxis(Hs, 2, 0))          # [n_p, n_c, n_c]
        rhs[e] = -np.einsum("jab,bj->aj", Hw, H[e][None, :] * r[e])
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()


def test_hadamard_conservation_adjoint_identity():
    """1^T H J = 0 per component for the conservative Hadamard form."""
    m, s, u = _setup(2, 1, form="hadamard", diss=True)
    J = dense_jacobian(s, u)
    H = m.H_all()
    for c in range(m.n_c):
        lam = np.zeros_like(u)
        lam[:, c, :] = H
        g = J.T @ lam.reshape(-1)
        assert np.abs(g).max() < 1e-12 * np.abs(J).max()


def test_complex_step_matches_central_differences():
    m, s, u = _setup(2, 2, diss=True)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(u.shape)
    lam = rng.standard_normal(u.shape)
    J = dense_jacobian(s, u)
    h = 1e-6
    fd = np.sum(lam * (s(u + h * v) - s(u - h * v))) / (2 * h)
    ad = lam.reshape(-1) @ J @ v.reshape(-1)
    assert abs(fd - ad) < 1e-7 * abs(ad)


def test_local_vjp_equals_dense():
    m, s, u = _setup(2, 1, diss=True)
    lam = np.random.default_rng(4).standard_normal(u.shape)
    from oracle.jacobian import vjp, vjp_elements
    full = vjp(s, u, lam)
    loc = vjp_elements(s, u, lam, [0, 3, 5])
    for e, g in loc.items():
        assert np.abs(g - full[e]).max() < 1e-13 * np.abs(full).max()
