"""Pins for the oracle's pointwise physics against identities the paper states
(Sec. 2.4, 3, 4, 4.4) and independent derivatives."""
import mpmath
import numpy as np
import pytest

from oracle import physics as ph

RNG = np.random.default_rng(12345)


def random_states(n, d, rng=RNG):
    rho = rng.uniform(0.5, 1.5, n)
    p = rng.uniform(0.5, 1.5, n)
    V = rng.uniform(-0.5, 0.5, (d, n))
    e = p / 0.4 + 0.5 * rho * np.sum(V * V, 0)
    return np.concatenate([rho[None], rho[None] * V, e[None]], 0)


def cstep_jacobian(fun, U, h=1e-30):
    """d fun / d U by complex step, fun: [n_c,...] -> [m,...]; returns [m, n_c, ...]."""
    nc = U.shape[0]
    cols = []
    for c in range(nc):
        Uc = U.astype(complex)
        Uc[c] += 1j * h
        cols.append(np.imag(fun(Uc)) / h)
    return np.stack(cols, 1)


GASES = [ph.Gas(beta=2.5), ph.Gas(beta=2.0), ph.Gas(beta=1.6)]


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("gas", GASES, ids=lambda g: f"beta{g.beta}")
def test_entropy_variables_are_gradient_of_entropy(d, gas):
    U = random_states(20, d)
    W = ph.entropy_vars(U, gas)
    dS = cstep_jacobian(lambda X: ph.entropy(X, gas)[None], U)[0]
    assert np.abs(W - dS).max() < 1e-13 * np.abs(W).max()


def test_beta_25_closed_form():
    """beta = 2.5, gamma = 1.4: alpha = -2.4, S = 2.5 rho^2.4 / p and
    W = rho^2.4/p^2 [6 p/rho - |V|^2/2, V, -1]."""
    gas = ph.Gas(beta=2.5)
    assert abs(gas.alpha + 2.4) < 1e-15
    U = random_states(10, 2)
    rho, V, p = ph.primitive(U, gas)
    S = 2.5 * rho ** 2.4 / p
    W = rho ** 2.4 / p ** 2 * np.concatenate([(6 * p / rho - 0.5 * np.sum(V * V, 0))[None], V, -np.ones((1, 10))])
    assert np.allclose(ph.entropy(U, gas), S, rtol=1e-14, atol=0)
    assert np.allclose(ph.entropy_vars(U, gas), W, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("gas", GASES, ids=lambda g: f"beta{g.beta}")
def test_inverse_map_and_symmetrizer(d, gas):
    U = random_states(20, d)
    W = ph.entropy_vars(U, gas)
    assert np.abs(ph.cons_from_entropy_vars(W, gas) - U).max() < 1e-13
    A0 = ph.dU_dW(U, gas)
    # A0 = (d^2 S / dU^2)^{-1} computed independently by complex step of W(U)
    Hs = cstep_jacobian(lambda X: ph.entropy_vars(X, gas), U)          # [n_c, n_c, n]
    prod = np.einsum("abn,bcn->acn", A0, Hs)
    eye = np.eye(d + 2)[:, :, None]
    assert np.abs(prod - eye).max() < 1e-12
    assert np.abs(A0 - np.swapaxes(A0, 0, 1)).max() < 1e-13 * np.abs(A0).max()
    # positive definite
    ev = np.linalg.eigvalsh(np.moveaxis(A0, 2, 0))
    assert (ev > 0).all()


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("gas", GASES, ids=lambda g: f"beta{g.beta}")
def test_flux_identities(d, gas):
    """A_i = dF/dU (complex step); A~_i symmetric; A~_i W = beta F (homogeneity
    in W); beta/(beta+1) W^T F = G; S = beta phi; G = beta psi (Sec. 3)."""
    U = random_states(15, d)
    W = ph.entropy_vars(U, gas)
    S = ph.entropy(U, gas)
    rho, V, p = ph.primitive(U, gas)
    for i in range(d):
        F = ph.flux(U, i, gas)
        A = ph.flux_jacobian(U, i, gas)
        Acs = cstep_jacobian(lambda X: ph.flux(X, i, gas), U)
        assert np.abs(A - Acs).max() < 1e-13 * np.abs(A).max()
        At = ph.symmetrized_jacobian(U, i, gas)
        assert np.abs(At - np.swapaxes(At, 0, 1)).max() < 1e-12 * np.abs(At).max()
        AtW = np.einsum("abn,bn->an", At, W)
        assert np.abs(AtW - gas.beta * F).max() < 1e-12 * np.abs(F).max()
        G = V[i] * S
        assert np.allclose(gas.beta / (gas.beta + 1) * np.sum(W * F, 0), G, rtol=1e-12, atol=1e-14)
        assert np.allclose(ph.potential_flux(U, i, gas) * gas.beta, G, rtol=1e-12, atol=1e-14)
        # homogeneity of degree beta of F(W) in W, through the inverse map
        eta = 1.7
        Fs = ph.flux(ph.cons_from_entropy_vars(eta * W, gas), i, gas)
        assert np.allclose(Fs, eta ** gas.beta * F, rtol=1e-12, atol=1e-13)
    assert np.allclose(gas.beta * ph.potential(U, gas), S, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("r", [7.0 / 12.0, 1.0 / 6.0, -0.3, 2.5])
def test_exponential_average_vs_mpmath(r):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7)
    a = rng.uniform(0.3, 3.0, 200)
    rel = np.concatenate([10.0 ** rng.uniform(-16, -0.3, 150), np.zeros(10), rng.uniform(0.01, 0.02, 40)])
    b = a[:200] * (1 + rel[:200] * rng.choice([-1, 1], 200))
    got = ph.exp_avg(a, b, r)
    for x, y, g in zip(a, b, got):
        X, Y = mpmath.mpf(float(x)), mpmath.mpf(float(y))
        if X == Y:
            ref = X ** (r - 1)
        else:
            ref = (X ** r - Y ** r) / (r * (X - Y))
        # series branch: a few ulp; direct branch: the difference a^r - b^r
        # cancels log10(1/|eps|) <= 2 digits, bound ~ 4 ulp / |eps|
        eps = abs((x - y) / (x + y))
        tol = 4e-15 if eps <= 1e-2 else 4 * 2.2e-16 / eps + 4e-15
        assert abs(g - float(ref)) <= tol * abs(float(ref))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("gas", GASES, ids=lambda g: f"beta{g.beta}")
def test_sjogreen_yee_flux(d, gas):
    """Consistency F*(U,U) = F(U), symmetry, Tadmor's condition
    (W'' - W')^T F*_i(U', U'') = psi'' - psi' (Sec. 4)."""
    Ua = random_states(30, d)
    Ub = random_states(30, d)
    Fab = ph.sy_flux(Ua, Ub, gas)
    Fba = ph.sy_flux(Ub, Ua, gas)
    assert np.abs(Fab - Fba).max() == 0.0
    Faa = ph.sy_flux(Ua, Ua, gas)
    Wa, Wb = ph.entropy_vars(Ua, gas), ph.entropy_vars(Ub, gas)
    for i in range(d):
        F = ph.flux(Ua, i, gas)
        assert np.abs(Faa[i] - F).max() < 1e-13 * np.abs(F).max()
        lhs = np.sum((Wb - Wa) * Fab[i], 0)
        rhs = ph.potential_flux(Ub, i, gas) - ph.potential_flux(Ua, i, gas)
        assert np.abs(lhs - rhs).max() < 1e-13
    # nearly equal states (series branch of the exponential average)
    Uc = Ua * (1 + 1e-9 * np.random.default_rng(1).standard_normal(Ua.shape))
    Fac = ph.sy_flux(Ua, Uc, gas)
    Wc = ph.entropy_vars(Uc, gas)
    for i in range(d):
        lhs = np.sum((Wc - Wa) * Fac[i], 0)
        rhs = ph.potential_flux(Uc, i, gas) - ph.potential_flux(Ua, i, gas)
        assert np.abs(lhs - rhs).max() < 1e-14


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("gas", GASES[:2], ids=lambda g: f"beta{g.beta}")
def test_dissipation_consistency_and_eigen(d, gas):
    """At equal states X S X^T = dU/dW (Sec. 4.5, consistency condition) and
    X diagonalises the normal flux Jacobian with |Lambda|; the operator is
    symmetric positive semidefinite and invariant under n -> -n."""
    rng = np.random.default_rng(3)
    U = random_states(8, d, rng)
    for k in range(U.shape[1]):
        n = rng.standard_normal(d)
        n /= np.linalg.norm(n)
        u = U[:, k]
        A0 = ph.dU_dW(u, gas)
        M = ph.dissipation_matrix(u, u, n, gas)
        An = sum(n[i] * ph.flux_jacobian(u, i, gas) for i in range(d))
        # independent route: |A_n| from a numerical eigen-decomposition, and
        # |A_n| A0 = X |Lambda| X^{-1} A0 = X |Lambda| S X^T when X S X^T = A0
        ev, R = np.linalg.eig(An)
        absAn = (R * np.abs(ev.real)[None, :]) @ np.linalg.inv(R)
        ref = absAn.real @ A0
        assert np.abs(M - ref).max() < 1e-11 * np.abs(ref).max()
        M2 = ph.dissipation_matrix(u, u, -n, gas)
        assert np.abs(M - M2).max() < 1e-12 * np.abs(M).max()
    # distinct states: symmetric PSD and n -> -n invariant
    Ub = random_states(8, d, rng)
    for k in range(U.shape[1]):
        n = rng.standard_normal(d)
        n /= np.linalg.norm(n)
        M = ph.dissipation_matrix(U[:, k], Ub[:, k], n, gas)
        assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > -1e-12 * np.abs(M).max()
        assert np.abs(M - ph.dissipation_matrix(U[:, k], Ub[:, k], -n, gas)).max() < 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("d", [2, 3])
def test_viscous_flux_against_primitive_derivatives(d):
    """F^V from a conservative gradient equals the textbook stress and heat
    flux computed from directional derivatives of analytic primitive fields."""
    gas = ph.Gas(mu=0.013, Pr=0.71, R=1.0)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((d + 2, d))

    def prim(x):
        rho = 1.1 + 0.1 * np.sin(a[0] @ x)
        V = [0.2 * np.cos(a[1 + k] @ x) for k in range(d)]
        p = 0.9 + 0.1 * np.cos(a[d + 1] @ x)
        return rho, V, p

    def cons(x):
        rho, V, p = prim(x)
        e = p / 0.4 + 0.5 * rho * sum(v * v for v in V)
        return np.array([rho] + [rho * v for v in V] + [e])

    x0 = rng.standard_normal(d)
    h = 1e-30
    grad_prim = []
    gradU = []
    for j in range(d):
        xc = x0.astype(complex)
        xc[j] += 1j * h
        rho, V, p = prim(xc)
        grad_prim.append((np.imag(rho) / h, [np.imag(v) / h for v in V], np.imag(p) / h))
        gradU.append(np.imag(cons(xc)) / h)
    U = cons(x0)
    FV = ph.viscous_flux(U, np.array(gradU), gas)
    rho, V, p = prim(x0)
    T = p / rho
    kappa = gas.mu * 1.4 / (0.4 * 0.71)
    for i in range(d):
        div = sum(grad_prim[k][1][k] for k in range(d))
        tau = [gas.mu * (grad_prim[j][1][i] + grad_prim[i][1][j] - (2 / 3 if i == j else 0) * div) for j in range(d)]
        dT = (grad_prim[i][2] - T * grad_prim[i][0]) / rho
        ref = np.array([0.0] + tau + [sum(V[j] * tau[j] for j in range(d)) + kappa * dT])
        assert np.abs(FV[i] - ref).max() < 1e-14
