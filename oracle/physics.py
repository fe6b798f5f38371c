"""Pointwise Euler / Navier-Stokes quantities (ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

All functions take state arrays with the component axis first, U[n_c, ...]
(n_c = d + 2: rho, rho V_1..rho V_d, e), vectorised over trailing axes, and
accept complex input so that complex-step derivatives of the whole residual
are possible (real-part comparisons, an analytic |.|).

Sources in the paper:
  fluxes, EOS ........................ Sec. 2.2 (governing equations)
  Harten entropy S_H, beta, alpha ..... Sec. 2.4 (eq. harten entropy)
  entropy variables W ................. Sec. 3 (eq. harten entropy variables)
  U(W): temperature T(W), W_nc ........ Sec. 3 (eq. T in W, eq. W5)
  potentials phi, psi ................. Sec. 2.4 (eqs. phi = wTu - s, psi = wTf - g)
  Sjogreen-Yee two-point flux ......... Sec. 4 (eqs. param vector, avg
                                        arithmetic / exponential, flux entries)
  matrix interface dissipation ........ Sec. 4.5 (intermediate states, S-hat,
                                        |Lambda|, X-hat)
  viscous flux ........................ Sec. 2.2 (tau, heat flux kappa dT/dx)

Readings of the paper taken here:
  * exponential average near equal arguments: series in eps=(a-b)/(a+b)
    for |eps| <= 1e-2, direct formula otherwise;
  * 3D eigenvectors X-hat: the two printed shear columns are replaced by
    orthonormal tangents (0, t, V-hat.t) (the printed pair is neither
    orthonormal nor defined for n = (0, +-1, 0));
  * Jacobians dU/dW are formed analytically through the primitive variables
    (dU/dQ)(dW/dQ)^{-1}, a route independent of the temperature-derivative
    formula printed with a sign/factor error in Sec. 3.

Parity: pinned in tests/test_oracle_physics.py against identities the paper
states (W = dS/dU, A0 symmetric, A_i W = beta F, beta/(beta+1) W^T F = G,
S = beta phi, G = beta psi, two-point flux consistency/symmetry/Tadmor,
X S X^T = dU/dW and A_n X = X Lambda at equal states), against mpmath for the
exponential average, and the viscous flux against direct differentiation of
the primitive fields.
"""
from __future__ import annotations

import numpy as np


class Gas:
    """gamma and the split parameter beta (Sec. 2.4; Sec. 6.4, Robustness: beta = 2.5)."""

    def __init__(self, gamma=1.4, beta=2.5, mu=0.0, Pr=0.71, R=1.0, heat_flux=True):
        self.gamma = float(gamma)
        self.beta = float(beta)
        # beta = -(gamma + alpha)/(gamma - 1)
        self.alpha = -self.gamma - self.beta * (self.gamma - 1.0)
        self.mu = float(mu)
        self.Pr = float(Pr)
        self.R = float(R)
        self.heat_flux = bool(heat_flux)

    @property
    def kappa(self):
        # c_p mu / Pr with c_p = gamma R / (gamma - 1)
        if not self.heat_flux:
            return 0.0
        return self.mu * self.gamma * self.R / ((self.gamma - 1.0) * self.Pr)


def cabs(z):
    """|z| that is complex-step safe (sign of the real part)."""
    z = np.asarray(z)
    if np.iscomplexobj(z):
        return z * np.sign(z.real)
    return np.abs(z)


def primitive(U, gas):
    d = U.shape[0] - 2
    rho = U[0]
    V = U[1:1 + d] / rho
    p = (gas.gamma - 1.0) * (U[d + 1] - 0.5 * rho * np.sum(V * V, axis=0))
    return rho, V, p


def entropy(U, gas):
    """Harten entropy S_H = beta rho (p rho^-gamma)^(1/(alpha+gamma))."""
    rho, V, p = primitive(U, gas)
    return gas.beta * rho * (p * rho ** (-gas.gamma)) ** (1.0 / (gas.alpha + gas.gamma))


def entropy_vars(U, gas):
    """W = (rho/p)(p rho^-gamma)^(1/(alpha+gamma)) [-alpha/(gamma-1) p/rho - |V|^2/2, V, -1]."""
    rho, V, p = primitive(U, gas)
    g, a = gas.gamma, gas.alpha
    z1 = (rho / p) * (p * rho ** (-g)) ** (1.0 / (a + g))
    first = -a / (g - 1.0) * p / rho - 0.5 * np.sum(V * V, axis=0)
    return np.concatenate([(z1 * first)[None], z1[None] * V, (-z1)[None]], 0)


def cons_from_entropy_vars(W, gas):
    """Inverse map U(W): V = -W_V / W_nc; p/rho from the temperature formula
    (T = p/(rho R)); rho from the W_nc formula of Sec. 3."""
    d = W.shape[0] - 2
    g, a = gas.gamma, gas.alpha
    Wn = W[d + 1]
    WV = W[1:1 + d]
    V = -WV / Wn
    theta = (g - 1.0) * (2.0 * W[0] * Wn - np.sum(WV * WV, axis=0)) / (2.0 * a * Wn * Wn)
    # -W_nc = theta^((1-a-g)/(a+g)) rho^((1-g)/(a+g))
    rho = (-Wn * theta ** (-(1.0 - a - g) / (a + g))) ** ((a + g) / (1.0 - g))
    p = rho * theta
    e = p / (g - 1.0) + 0.5 * rho * np.sum(V * V, axis=0)
    return np.concatenate([rho[None], rho[None] * V, e[None]], 0)


def flux(U, i, gas):
    """Inviscid flux F^{I(i)}(U)."""
    d = U.shape[0] - 2
    rho, V, p = primitive(U, gas)
    out = [rho * V[i]]
    for j in range(d):
        out.append(rho * V[i] * V[j] + (p if j == i else 0.0))
    out.append((U[d + 1] + p) * V[i])
    return np.stack(out, 0)


def flux_jacobian(U, i, gas):
    """A_i = dF^{I(i)}/dU in closed form (textbook), shape [n_c, n_c, ...]."""
    d = U.shape[0] - 2
    nc = d + 2
    g = gas.gamma
    rho, V, p = primitive(U, gas)
    e = U[d + 1]
    q2 = np.sum(V * V, axis=0)
    H = (e + p) / rho
    shape = (nc, nc) + np.shape(rho)
    A = np.zeros(shape, dtype=np.result_type(U, 1.0))
    # mass row
    A[0, 1 + i] = 1.0
    # momentum rows
    for j in range(d):
        A[1 + j, 0] = -V[i] * V[j] + (0.5 * (g - 1.0) * q2 if j == i else 0.0)
        for k in range(d):
            val = 0.0
            if k == i:
                val = val + V[j]
            if k == j:
                val = val + V[i]
            if j == i:
                val = val - (g - 1.0) * V[k]
            A[1 + j, 1 + k] = val * np.ones_like(rho)
        A[1 + j, nc - 1] = (g - 1.0) if j == i else 0.0
    # energy row
    A[nc - 1, 0] = V[i] * (0.5 * (g - 1.0) * q2 - H)
    for k in range(d):
        A[nc - 1, 1 + k] = H * (1.0 if k == i else 0.0) - (g - 1.0) * V[i] * V[k]
    A[nc - 1, nc - 1] = g * V[i]
    return A


def _move(M):
    """[n, n, ...] -> [..., n, n] for batched linear algebra."""
    return np.moveaxis(np.moveaxis(M, 0, -1), 0, -1)


def _unmove(M):
    return np.moveaxis(np.moveaxis(M, -1, 0), -1, 0)


def dU_dW(U, gas):
    """A0 = dU/dW = (dU/dQ) (dW/dQ)^{-1} with Q = (rho, V, p), shape [n_c,n_c,...]."""
    d = U.shape[0] - 2
    nc = d + 2
    g, a = gas.gamma, gas.alpha
    rho, V, p = primitive(U, gas)
    dt = np.result_type(U, 1.0)
    sh = (nc, nc) + np.shape(rho)
    dUdQ = np.zeros(sh, dtype=dt)
    dUdQ[0, 0] = 1.0
    for j in range(d):
        dUdQ[1 + j, 0] = V[j]
        dUdQ[1 + j, 1 + j] = rho
        dUdQ[nc - 1, 1 + j] = rho * V[j]
    dUdQ[nc - 1, 0] = 0.5 * np.sum(V * V, axis=0)
    dUdQ[nc - 1, nc - 1] = 1.0 / (g - 1.0)
    # W = z1 * v, z1 = rho^m p^n, v = [-a/(g-1) p/rho - |V|^2/2, V, -1]
    m = a / (a + g)
    n = (1.0 - a - g) / (a + g)
    z1 = rho ** m * p ** n
    v0 = -a / (g - 1.0) * p / rho - 0.5 * np.sum(V * V, axis=0)
    v = [v0] + [V[j] for j in range(d)] + [-np.ones_like(rho)]
    dvdQ = np.zeros(sh, dtype=dt)
    dvdQ[0, 0] = a / (g - 1.0) * p / (rho * rho)
    dvdQ[0, nc - 1] = -a / ((g - 1.0) * rho)
    for j in range(d):
        dvdQ[0, 1 + j] = -V[j]
        dvdQ[1 + j, 1 + j] = 1.0
    dz = [m * z1 / rho] + [np.zeros_like(rho)] * d + [n * z1 / p]
    dWdQ = np.zeros(sh, dtype=dt)
    for r in range(nc):
        for c in range(nc):
            dWdQ[r, c] = z1 * dvdQ[r, c] + v[r] * dz[c]
    A0 = np.linalg.solve(_move(dWdQ).swapaxes(-1, -2), _move(dUdQ).swapaxes(-1, -2)).swapaxes(-1, -2)
    return _unmove(A0)


def symmetrized_jacobian(U, i, gas):
    """A~_i = A_i A0 (Sec. 2.4, eq. symmetric coefficients)."""
    A = _move(flux_jacobian(U, i, gas))
    A0 = _move(dU_dW(U, gas))
    return _unmove(A @ A0)


def potential(U, gas):
    """phi = W^T U - S."""
    W = entropy_vars(U, gas)
    return np.sum(W * U, axis=0) - entropy(U, gas)


def potential_flux(U, i, gas):
    """psi^(i) = W^T F^(i) - G^(i), G^(i) = V_i S."""
    W = entropy_vars(U, gas)
    rho, V, p = primitive(U, gas)
    return np.sum(W * flux(U, i, gas), axis=0) - V[i] * entropy(U, gas)


def exp_avg(a, b, r):
    """Exponential average {u^{r-1}}_e = (a^r - b^r)/(r (a - b)) (Sec. 4).

    For |eps| <= 1e-2, eps = (a-b)/(a+b), m = (a+b)/2, the equivalent series
    m^{r-1} [1 + sum_{k=1..4} C(r,2k+1)/r eps^{2k}],
    C(r,2k+1)/r = (r-1)(r-2)...(r-2k)/(2k+1)!, is used (truncation < 1e-20)."""
    a = np.asarray(a)
    b = np.asarray(b)
    eps = (a - b) / (a + b)
    m = 0.5 * (a + b)
    coef = []
    c = 1.0
    for k in range(1, 5):
        c = c * (r - (2 * k - 1)) * (r - 2 * k) / ((2 * k) * (2 * k + 1))
        coef.append(c)
    e2 = eps * eps
    series = m ** (r - 1.0) * (1.0 + e2 * (coef[0] + e2 * (coef[1] + e2 * (coef[2] + e2 * coef[3]))))
    small = np.abs(np.real(eps)) <= 1e-2
    with np.errstate(divide="ignore", invalid="ignore"):
        direct = (a ** r - b ** r) / (r * (a - b))
    return np.where(small, series, direct)


def sy_param(U, gas):
    """Parameter vector z = [z1, V, p], z1 = (rho/p)(p rho^-gamma)^(1/(alpha+gamma))."""
    rho, V, p = primitive(U, gas)
    z1 = (rho / p) * (p * rho ** (-gas.gamma)) ** (1.0 / (gas.alpha + gas.gamma))
    return z1, V, p


def sy_flux(Uk, Uv, gas):
    """Sjogreen-Yee two-point flux F*_i(Uk, Uv) for i = 1..d, shape [d, n_c, ...]."""
    g, a = gas.gamma, gas.alpha
    z1k, Vk, pk = sy_param(Uk, gas)
    z1v, Vv, pv = sy_param(Uv, gas)
    d = Vk.shape[0]
    avg = lambda x, y: 0.5 * (x + y)
    r1 = -g / a                 # exponent of z1 in the averages
    r2 = (1.0 - g) / a          # exponent of p
    Ep = exp_avg(pk, pv, r2)    # {p^{(1-g-a)/a}}_e
    Ez = exp_avg(z1k, z1v, r1)  # {z1^{-(g+a)/a}}_e
    den = avg(z1k ** r1, z1v ** r1) * Ep
    out = []
    q2avg = avg(np.sum(Vk * Vk, axis=0), np.sum(Vv * Vv, axis=0))
    Vav = [avg(Vk[j], Vv[j]) for j in range(d)]
    for i in range(d):
        f1 = avg(z1k * Vk[i], z1v * Vv[i]) / den
        comp = [f1]
        for j in range(d):
            comp.append(f1 * Vav[j] + (avg(pk, pv) if j == i else 0.0))
        en = g / (g - 1.0) * avg(pk ** r2, pv ** r2) * Ez + sum(v * v for v in Vav) - 0.5 * q2avg
        comp.append(f1 * en)
        out.append(np.stack(comp, 0))
    return np.stack(out, 0)


def _tangents(n):
    """Orthonormal tangents to the unit normal n (3D)."""
    n = np.asarray(n, dtype=np.float64)
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = np.cross(a, n)
    t1 = t1 / np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    return [t1, t2]


def dissipation_matrix(Uk, Uv, n, gas):
    """X-hat |Lambda| S-hat X-hat^T at the intermediate state of one facet
    node pair (Sec. 4.5), for unit normal n (real, shape [d]); states are
    single nodes (shape [n_c]).  Returns [n_c, n_c]."""
    g, a = gas.gamma, gas.alpha
    z1k, Vk, pk = sy_param(Uk, gas)
    z1v, Vv, pv = sy_param(Uv, gas)
    d = Vk.shape[0]
    nc = d + 2
    r1 = -g / a
    r2 = (1.0 - g) / a
    Ep = exp_avg(pk, pv, r2)
    Ez = exp_avg(z1k, z1v, r1)
    D = 0.5 * (z1k ** r1 + z1v ** r1) * Ep
    z1a = 0.5 * (z1k + z1v)
    rho_h = z1a / D
    V_h = np.array([0.5 * (z1k * Vk[i] + z1v * Vv[i]) / z1a for i in range(d)])
    p_h = 0.5 * (pk + pv)
    theta = rho_h / (p_h * D)
    eta = 1.0 / (z1a * Ez * Ep)
    ah = np.sqrt(g * p_h / rho_h)
    Vn = sum(V_h[i] * n[i] for i in range(d))
    q2 = sum(V_h[i] * V_h[i] for i in range(d))
    Hh = ah * ah / (g - 1.0) + 0.5 * q2
    dt = np.result_type(Uk, Uv, 1.0)
    X = np.zeros((nc, nc), dtype=dt)
    # acoustic (-)
    X[0, 0] = 1.0
    for i in range(d):
        X[1 + i, 0] = V_h[i] - ah * n[i]
    X[nc - 1, 0] = Hh - ah * Vn
    # entropy
    X[0, 1] = 1.0
    for i in range(d):
        X[1 + i, 1] = V_h[i]
    X[nc - 1, 1] = 0.5 * q2
    # shear
    if d == 2:
        tans = [np.array([n[1], -n[0]])]
    else:
        tans = _tangents(n)
    for s, t in enumerate(tans):
        for i in range(d):
            X[1 + i, 2 + s] = t[i]
        X[nc - 1, 2 + s] = sum(V_h[i] * t[i] for i in range(d))
    # acoustic (+)
    X[0, nc - 1] = 1.0
    for i in range(d):
        X[1 + i, nc - 1] = V_h[i] + ah * n[i]
    X[nc - 1, nc - 1] = Hh + ah * Vn
    Sd = [theta / (2 * g), (g - 1.0) * (g + a) * theta / (g * a)] + [eta] * (d - 1) + [theta / (2 * g)]
    Ld = [cabs(Vn - ah), cabs(Vn)] + [cabs(Vn)] * (d - 1) + [cabs(Vn + ah)]
    diag = np.array([Ld[c] * Sd[c] for c in range(nc)], dtype=dt)
    return (X * diag[None, :]) @ X.T


def dissipation_parts(Uk, Uv, n, gas):
    """X-hat, S-hat, |Lambda| and the flux Jacobian data of the intermediate
    state, for tests of consistency and the eigen-relation."""
    g, a = gas.gamma, gas.alpha
    z1k, Vk, pk = sy_param(Uk, gas)
    z1v, Vv, pv = sy_param(Uv, gas)
    d = Vk.shape[0]
    nc = d + 2
    r1 = -g / a
    r2 = (1.0 - g) / a
    Ep = exp_avg(pk, pv, r2)
    Ez = exp_avg(z1k, z1v, r1)
    D = 0.5 * (z1k ** r1 + z1v ** r1) * Ep
    z1a = 0.5 * (z1k + z1v)
    rho_h = z1a / D
    V_h = np.array([0.5 * (z1k * Vk[i] + z1v * Vv[i]) / z1a for i in range(d)])
    p_h = 0.5 * (pk + pv)
    theta = rho_h / (p_h * D)
    eta = 1.0 / (z1a * Ez * Ep)
    return dict(rho=rho_h, V=V_h, p=p_h, theta=theta, eta=eta)


def viscous_flux(U, gradU, gas):
    """F^{V(i)} for i = 1..d from the conservative state and its gradient.

    gradU[j] = dU/dx_j, shape [d, n_c, ...].  Returns [d, n_c, ...]:
      [0, tau_i1..tau_id, sum_j V_j tau_ij + kappa dT/dx_i],
      tau_ij = mu (dV_i/dx_j + dV_j/dx_i - 2/3 delta_ij div V),  T = p/(rho R)."""
    d = U.shape[0] - 2
    g = gas.gamma
    rho, V, p = primitive(U, gas)
    T = p / (rho * gas.R)
    drho = [gradU[j][0] for j in range(d)]
    dV = [[(gradU[j][1 + k] - V[k] * drho[j]) / rho for j in range(d)] for k in range(d)]  # dV[k][j]
    dp = []
    for j in range(d):
        kin = sum(V[k] * dV[k][j] for k in range(d))
        dp.append((g - 1.0) * (gradU[j][d + 1] - 0.5 * np.sum(V * V, axis=0) * drho[j] - rho * kin))
    dT = [(dp[j] - gas.R * T * drho[j]) / (rho * gas.R) for j in range(d)]
    div = sum(dV[k][k] for k in range(d))
    out = []
    for i in range(d):
        tau = [gas.mu * (dV[i][j] + dV[j][i] - (2.0 / 3.0 if i == j else 0.0) * div) for j in range(d)]
        en = sum(V[j] * tau[j] for j in range(d)) + gas.kappa * dT[i]
        out.append(np.stack([np.zeros_like(rho)] + tau + [en], 0))
    return np.stack(out, 0)
