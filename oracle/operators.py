"""Reference-element diagonal-E SBP operators (ORACLE: test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

The paper prints no operator; Def. 1 and Sec. 2.1 fix what an operator must
satisfy, and the node counts it quotes for tetrahedra are context only.  An
operator of degree p on the reference simplex is built here as follows
(Sec. 2.1, "diagonal H and E" paragraph):

  * facet nodes: a positive, symmetric facet quadrature of degree >= 2p with
    points strictly inside each facet (triangle edges: (p+1)-point
    Gauss-Legendre; tetrahedron faces: a symmetric triangle rule), so each
    facet node belongs to exactly one facet and E is diagonal;
  * volume nodes: the facet nodes plus symmetric interior orbits whose
    positions and positive weights make H a quadrature of degree 2p-1;
  * E_l = sum_f R_f^T B_f N_{l,f} R_f (diagonal);
  * S_l = the minimum-Frobenius-norm skew matrix with S_l V = H V_l - E_l V / 2
    (V: Vandermonde of P^p, V_l its l-derivative), Q_l = S_l + E_l / 2,
    D_l = H^{-1} Q_l.

The node-set table below (orbit types and the starting guesses of their
parameters, node ordering) is an interface shared with the HIP library by
convention; both sides solve for the exact parameters on their own.

Node ordering: facet 0 nodes, facet 1 nodes, ..., then interior nodes.
Facet f is opposite vertex f.  Triangle facet f runs from vertex (f+1)%3 to
vertex (f+2)%3 with Gauss-Legendre parameters in ascending order.  A
tetrahedron face f uses the other three vertices in ascending order (a<b<c)
and the face-rule points (la, lb, lc) orbit by orbit.  Every orbit lists its
distinct permutations of barycentric coordinates in ascending lexicographic
order.

Parity: pinned by Def. 1 (tests/test_oracle_operators.py): SBP property
Q+Q^T=E, exactness of D on P^p, positivity of H and of facet weights,
exactness of H (degree 2p-1) and of facet rules (degree 2p).
"""
from __future__ import annotations

import functools
import itertools
from math import factorial

import mpmath
import numpy as np
from scipy.optimize import least_squares

# Orbit specifications.  Face rules live on a 2-simplex (barycentric triple);
# volume orbits on the element.  Each entry: (kind, starting guess).
#   '1'   centroid                        no parameter
#   '3'   (a, a, 1-2a)                    [a]
#   '6'   (a, b, 1-a-b)                   [a, b]
#   '12'  (a, a, b, 1-2a-b)  (tet)        [a, b]
FACE_RULES = {   # tetrahedron faces, degree 2p
    1: [("3", [1.0 / 6.0])],
    2: [("3", [0.4459]), ("3", [0.0916])],
    3: [("3", [0.2493]), ("3", [0.0631]), ("6", [0.0531, 0.3104])],
}
TRI_INTERIOR = {  # triangle interior orbits, volume degree 2p-1
    1: [],
    2: [("1", [])],
    3: [("6", [0.2288, 0.1871])],
    4: [("1", []), ("3", [0.1394]), ("3", [0.4384])],
}
TET_INTERIOR = {  # tetrahedron interior orbits
    1: [],
    2: [("1", [])],
    3: [("12", [0.1910, 0.1173])],
}
SUPPORTED = {2: (1, 2, 3, 4), 3: (1, 2, 3)}


def _perms(t):
    return sorted(set(itertools.permutations(t)))


def _orbit(kind, x, nbary):
    if kind == "1":
        return [tuple([1.0 / nbary] * nbary)]
    if kind == "3":
        a = x[0]
        return _perms((a, a, 1.0 - 2.0 * a))
    if kind == "6":
        a, b = x
        return _perms((a, b, 1.0 - a - b))
    if kind == "12":
        a, b = x
        return _perms((a, a, b, 1.0 - 2.0 * a - b))
    raise ValueError(kind)


def _npar(kind):
    return {"1": 0, "3": 1, "6": 2, "12": 2}[kind]


def _monomials(deg, dim):
    if dim == 2:
        return [(a, b) for a in range(deg + 1) for b in range(deg + 1 - a)]
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a)
            for c in range(deg + 1 - a - b)]


def _simplex_moment(e):
    """Integral of prod x_i^{e_i} over the unit reference simplex."""
    s = sum(e)
    num = 1.0
    for k in e:
        num *= factorial(k)
    return num / factorial(s + len(e))


def _eval_monomials(X, deg):
    dim = X.shape[1]
    return np.array([np.prod([X[:, i] ** m[i] for i in range(dim)], axis=0)
                     for m in _monomials(deg, dim)])


def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0,1], ascending points, weights sum 1.
    numpy's nodes are polished by Newton on P_n in 40-digit arithmetic and
    rounded, so the rule is the correctly rounded one."""
    t, _ = np.polynomial.legendre.leggauss(n)
    with mpmath.workdps(40):
        ts, ws = [], []
        for x0 in t:
            x = mpmath.mpf(float(x0))
            for _ in range(50):
                pn, pm = mpmath.legendre(n, x), mpmath.legendre(n - 1, x)
                dp = n * (x * pn - pm) / (x * x - 1)
                dx = pn / dp
                x -= dx
                if abs(dx) < mpmath.mpf("1e-38"):
                    break
            pn, pm = mpmath.legendre(n, x), mpmath.legendre(n - 1, x)
            dp = n * (x * pn - pm) / (x * x - 1)
            ts.append(float((x + 1) / 2))
            ws.append(float(1 / ((1 - x * x) * dp * dp)))
    order = np.argsort(ts)
    return np.array(ts)[order], np.array(ws)[order]


def _solve_orbit_rule(fixed_pts, fixed_gid, n_fixed_groups, orbits, deg, dim):
    """Find interior orbit parameters and group weights so that the rule
    (fixed points + orbits) integrates all monomials of degree <= deg over the
    reference simplex.  Weights enter linearly and are eliminated by least
    squares; parameters by nonlinear least squares from the starting guesses."""
    nbary = dim + 1
    mom = np.array([_simplex_moment(m) for m in _monomials(deg, dim)])
    x0 = np.array([v for _, g in orbits for v in g], dtype=np.float64)

    def assemble(x):
        pts = list(fixed_pts)
        gid = list(fixed_gid)
        k = 0
        g = n_fixed_groups
        for kind, _ in orbits:
            n = _npar(kind)
            o = _orbit(kind, x[k:k + n], nbary)
            k += n
            pts += [list(q) for q in o]
            gid += [g] * len(o)
            g += 1
        P = np.array(pts, dtype=np.float64)
        return P, np.array(gid), g

    def group_matrix(x):
        P, gid, ng = assemble(x)
        Vm = _eval_monomials(P[:, 1:], deg)
        G = np.stack([Vm[:, gid == g].sum(axis=1) for g in range(ng)], 1)
        return G

    def resid(x):
        G = group_matrix(x)
        w = np.linalg.lstsq(G, mom, rcond=None)[0]
        return G @ w - mom

    if x0.size:
        x = least_squares(resid, x0, xtol=1e-15, ftol=1e-15, gtol=1e-15).x
        x = _polish_mp(fixed_pts, fixed_gid, n_fixed_groups, orbits, deg, dim, x,
                       np.linalg.lstsq(group_matrix(x), mom, rcond=None)[0])
    else:
        x = x0
    # points from the rounded parameters in double arithmetic; weights by a
    # 40-digit least-squares solve for exactly these points, then rounded
    P, gid, ng = assemble(x)
    Vm = _eval_monomials(P[:, 1:], deg)
    G = np.stack([Vm[:, gid == g].sum(axis=1) for g in range(ng)], 1)
    with mpmath.workdps(40):
        Gm = mpmath.matrix(len(mom), ng)
        mons = _monomials(deg, dim)
        for g in range(ng):
            for q, m in enumerate(mons):
                acc = mpmath.mpf(0)
                for row in P[gid == g]:
                    t = mpmath.mpf(1)
                    for i in range(dim):
                        t *= mpmath.mpf(float(row[1 + i])) ** m[i]
                    acc += t
                Gm[q, g] = acc
        mm = mpmath.matrix([_simplex_moment_mp(m) for m in mons])
        wm = mpmath.lu_solve(Gm.T * Gm, Gm.T * mm)
        w = np.array([float(wm[g]) for g in range(ng)])
    return P, w[gid], x, np.abs(G @ w - mom).max()


def _simplex_moment_mp(e):
    num = mpmath.mpf(1)
    for k in e:
        num *= mpmath.factorial(k)
    return num / mpmath.factorial(sum(e) + len(e))


def _polish_mp(fixed_pts, fixed_gid, n_fixed_groups, orbits, deg, dim, x, w):
    """Gauss-Newton on the full moment system (parameters and group weights)
    in 40-digit arithmetic; returns the parameters rounded to doubles."""
    nbary = dim + 1
    mons = _monomials(deg, dim)
    with mpmath.workdps(40):
        mom = [_simplex_moment_mp(m) for m in mons]
        fixed = [[mpmath.mpf(float(v)) for v in pt] for pt in fixed_pts]

        def orbit_mp(kind, prm):
            one = mpmath.mpf(1)
            if kind == "1":
                base = [one / nbary] * nbary
            elif kind == "3":
                base = [prm[0], prm[0], 1 - 2 * prm[0]]
            elif kind == "6":
                base = [prm[0], prm[1], 1 - prm[0] - prm[1]]
            else:
                base = [prm[0], prm[0], prm[1], 1 - 2 * prm[0] - prm[1]]
            return [list(q) for q in set(itertools.permutations(base))] if kind != "1" else [base]

        def residual(z):
            xs, ws = z[:len(x)], z[len(x):]
            groups = [[] for _ in range(n_fixed_groups)]
            for pt, g in zip(fixed, fixed_gid):
                groups[g].append(pt)
            k = 0
            for kind, _ in orbits:
                n = _npar(kind)
                groups.append(orbit_mp(kind, xs[k:k + n]))
                k += n
            out = []
            for q, m in enumerate(mons):
                s = -mom[q]
                for g, pts in enumerate(groups):
                    acc = mpmath.mpf(0)
                    for pt in pts:
                        t = mpmath.mpf(1)
                        for i in range(dim):
                            t *= pt[1 + i] ** m[i]
                        acc += t
                    s += ws[g] * acc
                out.append(s)
            return out

        z = [mpmath.mpf(float(v)) for v in x] + [mpmath.mpf(float(v)) for v in w]
        h = mpmath.mpf("1e-28")
        for _ in range(30):
            R = residual(z)
            J = mpmath.matrix(len(R), len(z))
            for j in range(len(z)):
                zz = list(z)
                zz[j] += h
                Rj = residual(zz)
                for q in range(len(R)):
                    J[q, j] = (Rj[q] - R[q]) / h
            Rm = mpmath.matrix([-r for r in R])
            dz = mpmath.lu_solve(J.T * J, J.T * Rm)
            z = [z[j] + dz[j] for j in range(len(z))]
            if max(abs(dz[j]) for j in range(len(z))) < mpmath.mpf("1e-34"):
                break
        return np.array([float(v) for v in z[:len(x)]])


def _face_rule(p):
    """Symmetric triangle rule of degree 2p (barycentric points, weights
    summing to one) for the faces of a degree-p tetrahedral operator."""
    P, w, x, res = _solve_orbit_rule([], [], 0, FACE_RULES[p], 2 * p, 2)
    return P, 2.0 * w, res    # weights of the unit-area rule


def _facet_vertices(dim):
    if dim == 2:
        return [((f + 1) % 3, (f + 2) % 3) for f in range(3)]
    return [tuple(i for i in range(4) if i != f) for f in range(4)]


def _ref_vertices(dim):
    return np.vstack([np.zeros(dim), np.eye(dim)])


@functools.lru_cache(maxsize=None)
def reference_operator(dim: int, p: int) -> dict:
    """Diagonal-E SBP operator of degree p on the reference triangle
    (0,0),(1,0),(0,1) or tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1).

    Returns a dict with
      nodes [n_p,dim], h [n_p] (diagonal of H), Q,S,D [dim,n_p,n_p],
      E [dim,n_p] (diagonal of E), facet_nodes [n_fac,n_f] (int),
      facet_w [n_fac,n_f] (reference facet quadrature weights, physical
      measure of the reference facet), facet_normal [n_fac,dim] (unit
      outward normals), and the solved rule parameters.
    """
    if p not in SUPPORTED[dim]:
        raise ValueError(f"no operator for dim={dim}, p={p}")
    nb = dim + 1
    fverts = _facet_vertices(dim)
    # facet rule on one facet, in the facet's own barycentric coordinates
    if dim == 2:
        t, wt = gauss_legendre01(p + 1)
        fbary = np.stack([1.0 - t, t], 1)
        fw = wt
        face_res = 0.0
    else:
        fbary, fw, face_res = _face_rule(p)
    n_f = len(fw)
    bary = []
    facet_nodes = []
    for f, vs in enumerate(fverts):
        idx = []
        for q in fbary:
            lam = [0.0] * nb
            for c, v in enumerate(vs):
                lam[v] = q[c]
            idx.append(len(bary))
            bary.append(lam)
        facet_nodes.append(idx)
    # group facet nodes by symmetry class (equal weights) for the volume solve:
    # nodes on different facets with the same facet-rule weight and the same
    # sorted barycentric multiset form one orbit of the element symmetry group.
    keys = {}
    gid = []
    for f in range(len(fverts)):
        for j in range(n_f):
            k = tuple(np.round(sorted(fbary[j]), 10))
            keys.setdefault(k, len(keys))
            gid.append(keys[k])
    orbits = TRI_INTERIOR[p] if dim == 2 else TET_INTERIOR[p]
    P, h, xint, vol_res = _solve_orbit_rule(bary, gid, len(keys), orbits, 2 * p - 1, dim)
    X = P[:, 1:]
    n_p = len(X)
    # reference facet area-normals: -d |T| grad(lambda_f)
    Vref = _ref_vertices(dim)
    vol_ref = 1.0 / factorial(dim)
    Tm = np.stack([Vref[i] - Vref[0] for i in range(1, dim + 1)], 1)  # columns
    grads = np.zeros((nb, dim))
    Tinv = np.linalg.inv(Tm)
    grads[1:] = Tinv                      # grad lambda_i = row i-1 of T^{-1}
    grads[0] = -Tinv.sum(axis=0)
    area_normal = -dim * vol_ref * grads  # [nb,dim]
    area = np.linalg.norm(area_normal, axis=1)
    facet_normal = area_normal / area[:, None]
    facet_w = np.array([fw * area[f] for f in range(nb)])
    E = np.zeros((dim, n_p))
    for f in range(nb):
        for j, m in enumerate(facet_nodes[f]):
            E[:, m] += facet_w[f, j] * facet_normal[f]
    # Vandermonde of P^p in centred coordinates and its derivatives; the basis
    # is orthonormalised (Gram-Schmidt in 40-digit arithmetic) before the
    # double-precision least-squares solve, which then works with a
    # well-conditioned system.  S is basis independent.
    c = np.full(dim, 1.0 / nb)
    mons = _monomials(p, dim)
    nm = len(mons)
    Hm = np.diag(h)
    Q = np.zeros((dim, n_p, n_p))
    S = np.zeros((dim, n_p, n_p))
    D = np.zeros((dim, n_p, n_p))
    with mpmath.workdps(40):
        Y = [[mpmath.mpf(float(X[r, i])) - mpmath.mpf(1) / nb for i in range(dim)] for r in range(n_p)]

        def mono(r, m):
            t = mpmath.mpf(1)
            for i in range(dim):
                t *= Y[r][i] ** m[i]
            return t

        def dmono(r, m, l):
            if m[l] == 0:
                return mpmath.mpf(0)
            t = mpmath.mpf(m[l])
            for i in range(dim):
                t *= Y[r][i] ** (m[i] - (1 if i == l else 0))
            return t
        Vm = mpmath.matrix(n_p, nm)
        for r in range(n_p):
            for k, m in enumerate(mons):
                Vm[r, k] = mono(r, m)
        # modified Gram-Schmidt: V T = Qo with orthonormal columns
        T = mpmath.eye(nm)
        Qo = Vm.copy()
        for k in range(nm):
            for j in range(k):
                proj = sum(Qo[r, j] * Qo[r, k] for r in range(n_p))
                for r in range(n_p):
                    Qo[r, k] -= proj * Qo[r, j]
                for q in range(nm):
                    T[q, k] -= proj * T[q, j]
            nrm = mpmath.sqrt(sum(Qo[r, k] ** 2 for r in range(n_p)))
            for r in range(n_p):
                Qo[r, k] /= nrm
            for q in range(nm):
                T[q, k] /= nrm
        Vo = np.array([[float(Qo[r, k]) for k in range(nm)] for r in range(n_p)])
        Ao = []
        for l in range(dim):
            Am = mpmath.matrix(n_p, nm)
            for r in range(n_p):
                for k, m in enumerate(mons):
                    Am[r, k] = mpmath.mpf(float(h[r])) * dmono(r, m, l) - mpmath.mpf(float(E[l][r])) / 2 * Vm[r, k]
            AT = Am * T
            Ao.append(np.array([[float(AT[r, k]) for k in range(nm)] for r in range(n_p)]))
    iu = np.triu_indices(n_p, 1)
    nsk = len(iu[0])
    for l in range(dim):
        V, A = Vo, Ao[l]
        # unknowns: s_ij (i<j); S = sum s_ij (e_i e_j^T - e_j e_i^T).
        # constraint rows: (S V)[r, k] = A[r, k].
        M = np.zeros((n_p * nm, nsk))
        for q, (i, j) in enumerate(zip(*iu)):
            # column of S V contributed by s_ij: row i gets +V[j,:], row j gets -V[i,:]
            M[i * nm:(i + 1) * nm, q] += V[j]
            M[j * nm:(j + 1) * nm, q] -= V[i]
        s = np.linalg.lstsq(M, A.reshape(-1), rcond=None)[0]
        Sl = np.zeros((n_p, n_p))
        Sl[iu] = s
        Sl = Sl - Sl.T
        S[l] = Sl
        Q[l] = Sl + 0.5 * np.diag(E[l])
        D[l] = Q[l] / h[:, None]
    return dict(dim=dim, p=p, n_p=n_p, n_f=n_f, nodes=X, h=h, Q=Q, S=S, D=D, E=E,
                facet_nodes=np.array(facet_nodes, dtype=np.int64), facet_w=facet_w,
                facet_normal=facet_normal, facet_bary=fbary,
                interior_params=xint, rule_residual=max(vol_res, face_res))
