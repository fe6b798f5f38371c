"""Pins for the oracle's relaxation RK4 step (Sec. 6.1)."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle import rrk
from oracle.geometry import OracleMesh
from oracle.residual import OracleScheme
from paper_2305_07181_amd import workloads as wl


def vortex_setup(p=2, n=4):
    desc = wl.vortex2d_mesh(n)
    m = OracleMesh(desc, p)
    x = m.node_coords()
    rho, V, pr = wl.isentropic_vortex(np.moveaxis(x, 1, 0))
    u = np.moveaxis(wl.conservative(rho, V, pr), 0, 1)
    return m, u


@pytest.mark.parametrize("dissipation", [False, True])
def test_fully_discrete_entropy_equality(dissipation):
    """s(u_{n+1}) - s(u_n) = gamma e to roundoff; with an entropy-conservative
    residual e itself is O(dt^5)-small, so the entropy is conserved."""
    m, u = vortex_setup()
    s = OracleScheme(m, ph.Gas(), dissipation=dissipation)
    u = u * (1 + 0.01 * np.random.default_rng(0).standard_normal(u.shape))
    dt = s.timestep(u, 0.1)
    s0 = s.total_entropy(u)
    u1, gamma, d, e = rrk.rrk4_step(s, u, dt)
    s1 = s.total_entropy(u1)
    assert abs((s1 - s0) - gamma * e) < 64 * np.finfo(float).eps * abs(s0)
    assert 0.9 < gamma < 1.1
    if not dissipation:
        assert abs(s1 - s0) < 64 * np.finfo(float).eps * abs(s0)
    else:
        assert e < 0


def test_hybrid_switched_between_steps_conserves_entropy():
    """Thm. switching hybrid: the per-element choice of volume term may change
    from one RRK step to the next without loss of entropy conservation."""
    m, u = vortex_setup()
    u = u * (1 + 0.01 * np.random.default_rng(1).standard_normal(u.shape))
    rng = np.random.default_rng(5)
    s = OracleScheme(m, ph.Gas(), form="hybrid", element_form=rng.integers(0, 2, m.ne))
    dt = s.timestep(u, 0.1)
    s0 = s.total_entropy(u)
    for step in range(3):
        s.element_form = rng.integers(0, 2, m.ne)
        u, gamma, d, e = rrk.rrk4_step(s, u, dt)
        assert 0.9 < gamma < 1.1
    s1 = s.total_entropy(u)
    assert abs(s1 - s0) < 3 * 64 * np.finfo(float).eps * abs(s0)


def test_gamma_tends_to_one():
    """gamma_n = 1 + O(dt^p') as dt -> 0 (relaxation leaves RK4 order intact)."""
    m, u = vortex_setup()
    s = OracleScheme(m, ph.Gas(), dissipation=True)
    u = u * (1 + 0.01 * np.random.default_rng(1).standard_normal(u.shape))
    dt0 = s.timestep(u, 0.2)
    devs = []
    for k in range(3):
        _, gamma, _, _ = rrk.rrk4_step(s, u, dt0 / 2 ** k)
        devs.append(abs(gamma - 1))
    assert devs[0] > devs[1] > devs[2]
    assert np.log2(devs[1] / devs[2]) > 2.0


def test_rk4_tableau_is_fourth_order():
    """On a linear scalar problem du/dt = lambda u the RK4 direction equals
    the 4th-order Taylor polynomial of exp(lambda dt) - 1 times u."""
    lam = -0.4

    class Sch:
        gas = ph.Gas()

        class mesh:
            @staticmethod
            def H_all():
                return np.ones((1, 1))

        def __call__(self, y):
            return lam * y
    sch = Sch()
    u = np.array([[[1.0], [1.0], [1.0], [3.0]]])
    dt = 0.3
    d, _ = rrk.rk4_direction(sch, u, dt)
    z = lam * dt
    expect = z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.allclose(d, expect * u, rtol=1e-15, atol=0)
