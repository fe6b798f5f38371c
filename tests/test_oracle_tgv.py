"""Kinetic energy of the viscous Taylor-Green study (Sec. 7.5) in the oracle,
pinned by closed forms.

With u0 = rho0 = L = 1 the initial velocity gives |V|^2 / 2 =
(1 + cos 2x3)(1 - cos 2x1 cos 2x2) / 8, whose box average is 1/8; the density
p / (R T0) = 1 + (cos 2x1 + cos 2x2)(cos 2x3 + 2) / (16 p0) adds the average of
(cos 2x1 + cos 2x2)(1 - cos 2x1 cos 2x2) times a function of x3 alone, which
vanishes by orthogonality.  So E_k(0) = 1/8 exactly for every Mach number."""
import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle.geometry import OracleMesh
from oracle.residual import OracleScheme
from paper_2305_07181_amd import workloads as wl


def _cons(m, fields):
    x = np.moveaxis(m.node_coords(), 1, 0)
    rho, V, p = fields(x)
    return np.ascontiguousarray(np.moveaxis(wl.conservative(rho, V, p), 0, 1))


def test_uniform_flow_kinetic_energy_is_exact():
    m = OracleMesh(wl.periodic_tet_mesh(2, 1.5), 2)
    rho0, V0 = 1.3, np.array([0.4, -0.7, 0.2])

    def fields(x):
        one = np.ones(x.shape[1:])
        return rho0 * one, V0[:, None, None] * one, 2.0 * one

    ek = OracleScheme(m, ph.Gas()).kinetic_energy(_cons(m, fields))
    assert abs(ek - 0.5 * rho0 * V0 @ V0 * 1.5 ** 3) <= 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_taylor_green_initial_kinetic_energy(p):
    """E_k of the nodal initial field tends to 1/8 as the grid is refined: on
    4^3 x 6 tetrahedra the diagonal norm of the periodic grid integrates the
    field's few Fourier modes (wavenumbers up to 4) exactly, to rounding."""
    errs = []
    for n in (2, 4):
        m = OracleMesh(wl.tgv_mesh(n), p)
        u = _cons(m, wl.taylor_green)
        ek = OracleScheme(m, ph.Gas()).kinetic_energy(u) / (2 * math.pi) ** 3
        errs.append(abs(ek - 0.125))
    assert errs[0] > 1e-4 and errs[1] <= 1e-13, errs
