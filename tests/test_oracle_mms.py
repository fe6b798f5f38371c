"""Pins for the oracle's manufactured solution and source (Sec. 7, manufactured
solution for the compressible Navier-Stokes equations): the source written
term by term agrees with fourth-order central differences of the oracle's
inviscid and viscous fluxes (physics.flux, physics.viscous_flux) applied to
the fields, a constant state has no source, and the paper's pressure gives
the total energy rho^2 when |V|^2 = d."""
import numpy as np
import pytest

from oracle import mms
from oracle import physics as ph

H = 1e-3
W4 = ((-2, 1.0 / 12.0), (-1, -8.0 / 12.0), (1, 8.0 / 12.0), (2, -1.0 / 12.0))


def _d4(fun, x, t, axis):
    """Fourth-order central difference of fun(x, t) along x_axis (axis < d) or t."""
    acc = 0.0
    for k, w in W4:
        if axis == "t":
            acc = acc + w * fun(x, t + k * H)
        else:
            xs = x.copy()
            xs[axis] = xs[axis] + k * H
            acc = acc + w * fun(xs, t)
    return acc / H


def _fd_source(x, t, gas, par, viscous):
    d = x.shape[0]
    U = lambda xx, tt: mms.state(xx, tt, gas, par)
    S = _d4(U, x, t, "t")
    for i in range(d):
        S = S + _d4(lambda xx, tt: ph.flux(U(xx, tt), i, gas), x, t, i)
    if viscous:
        def FV(xx, tt, i):
            grad = np.stack([_d4(U, xx, tt, j) for j in range(d)], 0)
            return ph.viscous_flux(U(xx, tt), grad, gas)[i]
        for i in range(d):
            S = S - _d4(lambda xx, tt: FV(xx, tt, i), x, t, i)
    return S


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("mu,heat", [(0.0, True), (0.01, True), (0.5, True), (0.5, False)])
def test_source_matches_flux_differences(d, mu, heat):
    rng = np.random.default_rng(7 + d)
    x = rng.uniform(-1.0, 1.0, (d, 12))
    gas = ph.Gas(mu=mu, Pr=0.71, R=1.0, heat_flux=heat)
    for par, t in ((mms.PAPER, 0.0), (mms.PAPER, 0.37), ((1.5, 0.3, -0.4, 0.7), 0.2)):
        S = mms.source(x, t, gas, par, viscous=mu > 0)
        Sf = _fd_source(x, t, gas, par, viscous=mu > 0)
        assert np.abs(S - Sf).max() < 1e-7 * max(1.0, np.abs(S).max()), np.abs(S - Sf).max()
    if mu > 0 and heat:
        # the heat-flux term is large enough here that dropping it fails the bar
        S_inv = mms.source(x, 0.37, gas, mms.PAPER, viscous=False)
        Sf = _fd_source(x, 0.37, gas, mms.PAPER, viscous=True)
        assert np.abs(S_inv - Sf).max() > 1e-4


def test_constant_state_has_no_source():
    x = np.random.default_rng(3).uniform(-1, 1, (3, 10))
    gas = ph.Gas(mu=0.01)
    S = mms.source(x, 0.5, gas, (2.0, 0.0, 0.6, 1.0))
    assert np.abs(S).max() < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_paper_fields_energy_is_rho_squared(d):
    """With V_i = 1 the paper's pressure makes the total energy rho^2; the
    primitive variables read back from the state are the fields."""
    x = np.random.default_rng(5).uniform(-1, 1, (d, 20))
    gas = ph.Gas()
    U = mms.state(x, 0.25, gas)
    rho = 2.0 + 0.1 * np.sin(np.pi * (x.sum(0) - 0.6 * 0.25))
    assert np.abs(U[d + 1] - rho ** 2).max() < 1e-14
    r, V, p = ph.primitive(U, gas)
    assert np.abs(r - rho).max() < 1e-15 and np.abs(V - 1.0).max() < 1e-14
    assert np.abs(p - 0.4 * (rho ** 2 - 0.5 * d * rho)).max() < 1e-14


def test_fields_periodic_with_period_two():
    x = np.random.default_rng(9).uniform(-1, 1, (3, 8))
    gas = ph.Gas(mu=0.01)
    for i in range(3):
        xs = x.copy()
        xs[i] += 2.0
        assert np.abs(mms.state(xs, 0.1, gas) - mms.state(x, 0.1, gas)).max() < 1e-13
        assert np.abs(mms.source(xs, 0.1, gas) - mms.source(x, 0.1, gas)).max() < 1e-12


def test_l2_error_of_exact_state_is_zero_and_scales():
    gas = ph.Gas()
    x = np.random.default_rng(2).uniform(-1, 1, (4, 2, 6))   # [ne, d, n_p]
    Hw = np.random.default_rng(3).uniform(0.1, 1.0, (4, 6))
    ue = np.moveaxis(mms.state(np.moveaxis(x, 1, 0), 0.3, gas), 0, 1)
    assert np.abs(mms.l2_error(ue, x, 0.3, Hw, gas)).max() == 0.0
    du = np.zeros_like(ue)
    du[:, 0, :] = 1e-3
    e = mms.l2_error(ue + du, x, 0.3, Hw, gas)
    assert abs(e[0] - 1e-6 * Hw.sum()) < 1e-9 * 1e-6 * Hw.sum() and np.abs(e[1:]).max() == 0.0


def test_source_keeps_discrete_solution_on_the_fields():
    """Relaxation RK4 of the oracle scheme with the source added at the stage
    times follows the manufactured fields to the spatial error; without the
    source (or with its sign flipped) the state leaves them by about dt |S|
    per step."""
    from oracle import rrk
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import workloads as wl
    gas = ph.Gas()
    m = OracleMesh(wl.mms_mesh2d(4), 3)
    sch = OracleScheme(m, gas)
    x = m.node_coords()                                      # [ne, d, n_p]
    xs = np.moveaxis(x, 1, 0)
    exact = lambda t: np.moveaxis(mms.state(xs, t, gas), 0, 1)
    src = lambda t: np.moveaxis(mms.source(xs, t, gas, viscous=False), 0, 1)
    H = m.H_all()
    dt, nstep = 2e-3, 3
    errs = {}
    for name, f in (("with", src), ("without", None), ("flipped", lambda t: -src(t))):
        u, t = exact(0.0), 0.0
        for _ in range(nstep):
            u, g, _, _ = rrk.rrk4_step(sch, u, dt, f, t)
            t += g * dt
        errs[name] = np.sqrt(mms.l2_error(u, x, t, H, gas).sum())
    drift = nstep * dt * np.sqrt(np.einsum("en,ecn->", H, src(0.0) ** 2))
    assert errs["with"] < 0.2 * drift, errs
    assert errs["without"] > 0.5 * drift and errs["flipped"] > 1.5 * drift, (errs, drift)


@pytest.mark.parametrize("dim,k", [(2, 4), (2, 13), (3, 4), (3, 10)])
def test_simplex_rule_integrates_monomials(dim, k):
    """The collapsed rule integrates every monomial of degree <= k exactly
    (a! b! [c!] / (a + b [+ c] + dim)! on the unit simplex)."""
    from math import factorial
    xq, wq = mms.simplex_rule(dim, k)
    rng = range(k + 1)
    for a in rng:
        for b in rng:
            for c in (range(k + 1) if dim == 3 else [0]):
                if a + b + c > k:
                    continue
                val = np.sum(wq * xq[:, 0] ** a * xq[:, 1] ** b * (xq[:, 2] ** c if dim == 3 else 1.0))
                ex = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + dim)
                assert abs(val - ex) <= 1e-14 * max(ex, 1e-3), (a, b, c, val, ex)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 4), (3, 1), (3, 3)])
def test_interp_matrix_reproduces_degree_p(dim, p):
    from oracle.operators import reference_operator
    op = reference_operator(dim, p)
    xq, _ = mms.simplex_rule(dim, 3 * p + 1)
    I = mms.interp_matrix(op["nodes"], op["h"], p, xq)
    rng = np.random.default_rng(p)
    coef = rng.standard_normal(dim + 1)
    f = lambda x: coef[0] + sum(coef[1 + i] * x[:, i] for i in range(dim)) ** p
    assert np.abs(I @ f(op["nodes"]) - f(xq)).max() < 1e-12
    assert np.abs(I.sum(axis=1) - 1.0).max() < 1e-13


@pytest.mark.parametrize("dim,p,curved", [(2, 1, False), (2, 3, False), (3, 2, False), (2, 1, True), (2, 4, True)])
def test_quadrature_norm_of_offset_is_box_volume(dim, p, curved):
    """u = (a field the interpolant reproduces) + c in one component: the
    integrated squared error is c^2 times the box volume 2^d.  On affine
    grids the field is a degree-p polynomial; on the curved 2D grid (which
    tiles the same box; its P2 Jacobian is integrated exactly) a constant."""
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import workloads as wl
    if dim == 3:
        desc = wl.mms_mesh3d(2)
    elif curved:
        desc = wl.mms_mesh2d(3)
    else:
        desc = wl.periodic_tri_mesh(3, 3, 2.0)
    m = OracleMesh(desc, p)
    q = 0 if curved else p
    poly = lambda x: np.stack([1.0 + 0.3 * x[0] ** q] + [0.5 * x[i] ** q for i in range(dim)]
                              + [2.0 + 0.1 * x[-1] ** q], 0)
    u = np.stack([poly(m.node_coords()[e]) for e in range(m.ne)], 0)
    c = 0.25
    u[:, 1, :] += c
    err = mms.l2_error_quadrature(u, m, poly)
    assert abs(err[1] - c * c * 2.0 ** dim) < 1e-12, err
    assert np.abs(np.delete(err, 1)).max() < 1e-24


@pytest.mark.parametrize("p", [1, 2, 3])
def test_quadrature_norm_of_nodal_fields_decays_at_p_plus_one(p):
    """The fields sampled at the nodes differ from the fields between the
    nodes by the interpolation error, which falls as h^(p+1)."""
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import workloads as wl
    gas = ph.Gas()
    errs = []
    for n in (6, 12):
        m = OracleMesh(wl.mms_mesh2d(n), p)
        xs = np.moveaxis(m.node_coords(), 1, 0)
        u = np.ascontiguousarray(np.moveaxis(mms.state(xs, 0.2, gas), 0, 1))
        errs.append(np.sqrt(mms.l2_error_quadrature(u, m, lambda x: mms.state(x, 0.2, gas)).sum()))
    rate = np.log(errs[0] / errs[1]) / np.log(2.0)
    assert p + 0.7 < rate < p + 1.5, (errs, rate)


def test_vortex3d_solves_the_euler_equations():
    """The 3D vortex of the accuracy study (with the reading of its garbled
    V_1 exponent) satisfies du/dt + div F = 0: fourth-order differences of
    the oracle's fluxes vanish to the difference error; the misread
    exponent (x1 - t)^2 in V_1 does not."""
    gas = ph.Gas()
    x = np.random.default_rng(4).uniform(-2.0, 2.0, (3, 16))
    U = lambda xx, tt: mms.vortex3d_state(xx, tt, gas)
    R = _d4(U, x, 0.3, "t")
    for i in range(3):
        R = R + _d4(lambda xx, tt: ph.flux(U(xx, tt), i, gas), x, 0.3, i)
    assert np.abs(R).max() < 1e-8, np.abs(R).max()
    assert np.abs(U(x, 0.3)[3]).max() == 0.0

    def misread(xx, tt):
        u = U(xx, tt)
        y = xx[1] - tt
        V1 = -0.4 * y * np.exp(0.5 * (1.0 - (xx[0] - tt) ** 2 - xx[0] ** 2))
        u2 = u.copy()
        u2[1] = u[0] * V1
        V = u2[1:4] / u[0]
        p = u[0] ** gas.gamma / gas.gamma
        u2[4] = p / (gas.gamma - 1.0) + 0.5 * u[0] * np.sum(V * V, 0)
        return u2
    R2 = _d4(misread, x, 0.3, "t")
    for i in range(3):
        R2 = R2 + _d4(lambda xx, tt: ph.flux(misread(xx, tt), i, gas), x, 0.3, i)
    assert np.abs(R2).max() > 1e-3
