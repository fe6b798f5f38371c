"""Pins for the oracle's reference SBP operators (Def. 1 and Sec. 2.1)."""
from math import factorial

import numpy as np
import pytest

from oracle.operators import SUPPORTED, reference_operator, gauss_legendre01

CASES = [(2, p) for p in SUPPORTED[2]] + [(3, p) for p in SUPPORTED[3]]


def monomials(deg, dim):
    if dim == 2:
        return [(a, b) for a in range(deg + 1) for b in range(deg + 1 - a)]
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a) for c in range(deg + 1 - a - b)]


def simplex_integral(e):
    num = 1.0
    for k in e:
        num *= factorial(k)
    return num / factorial(sum(e) + len(e))


def evalm(X, m):
    return np.prod([X[:, i] ** m[i] for i in range(X.shape[1])], axis=0)


def devalm(X, m, l):
    if m[l] == 0:
        return np.zeros(len(X))
    mm = list(m)
    mm[l] -= 1
    return m[l] * evalm(X, mm)


@pytest.mark.parametrize("dim,p", CASES)
def test_sbp_property_and_exactness(dim, p):
    op = reference_operator(dim, p)
    X = op["nodes"]
    for l in range(dim):
        Q, S, E = op["Q"][l], op["S"][l], op["E"][l]
        assert np.abs(S + S.T).max() == 0.0
        assert np.abs(Q + Q.T - np.diag(E)).max() < 1e-14
        scale = np.abs(op["D"][l]).max()
        for m in monomials(p, dim):
            err = np.abs(op["D"][l] @ evalm(X, m) - devalm(X, m, l)).max()
            assert err < 1e-13 * scale, (l, m, err)


@pytest.mark.parametrize("dim,p", CASES)
def test_norm_is_positive_quadrature_of_degree_2p_minus_1(dim, p):
    op = reference_operator(dim, p)
    h, X = op["h"], op["nodes"]
    assert (h > 0).all()
    for m in monomials(2 * p - 1, dim):
        assert abs(h @ evalm(X, m) - simplex_integral(m)) < 1e-14
    # nodes inside the closed element
    bary = np.concatenate([1 - X.sum(1, keepdims=True), X], 1)
    assert (bary > -1e-14).all()


@pytest.mark.parametrize("dim,p", CASES)
def test_facet_rules_and_E(dim, p):
    """E_l = sum_f R^T B N_l R: facet weights positive, facet rule exact to
    degree 2p on every facet, nodes on their facet, E integrates boundary
    products  p^T E_l q = closed-surface integral of P Q n_l  (Def. 1, item 3)."""
    op = reference_operator(dim, p)
    X = op["nodes"]
    nb = dim + 1
    bary = np.concatenate([1 - X.sum(1, keepdims=True), X], 1)
    assert (op["facet_w"] > 0).all()
    all_facet = np.concatenate(op["facet_nodes"])
    assert len(set(all_facet.tolist())) == len(all_facet)   # each facet node on one facet
    for f in range(nb):
        idx = op["facet_nodes"][f]
        assert np.abs(bary[idx, f]).max() < 1e-15
        # exactness on the facet: parametrise by the facet's barycentrics
        fb = op["facet_bary"]
        area = op["facet_w"][f].sum()
        if dim == 2:
            for k in range(2 * p + 1):
                quad = (op["facet_w"][f] / area) @ (fb[:, 1] ** k)
                assert abs(quad - 1.0 / (k + 1)) < 1e-14
        else:
            for m in monomials(2 * p, 2):
                quad = (op["facet_w"][f] / area) @ (fb[:, 1] ** m[0] * fb[:, 2] ** m[1])
                assert abs(quad - 2 * simplex_integral(m)) < 1e-14
    # closed surface: sum of E_l = 0; and E_l applied to x_l gives the volume
    vol = 1.0 / factorial(dim)
    for l in range(dim):
        assert abs(op["E"][l].sum()) < 1e-14
        assert abs(op["E"][l] @ X[:, l] - vol) < 1e-14


def test_gauss_legendre_closed_forms():
    t, w = gauss_legendre01(2)
    assert np.allclose(t, [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)], atol=1e-16, rtol=0)
    assert np.allclose(w, [0.5, 0.5], atol=1e-16, rtol=0)
    t, w = gauss_legendre01(3)
    assert np.allclose(t, [0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)], atol=2e-16, rtol=0)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=2e-16, rtol=0)


def _load_dunavant():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "triangle_rules.txt")
    rules = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        deg, *vals = line.split()
        rules.setdefault(int(deg), []).append([float(v) for v in vals])
    return rules


@pytest.mark.parametrize("p", [2, 3])
def test_tet_face_rules_match_published_symmetric_rules(p):
    """The face rule the oracle solves for is the published symmetric
    triangle rule of degree 2p (stored in tests/golden with its source)."""
    rules = _load_dunavant()[2 * p]
    op = reference_operator(3, p)
    fb = op["facet_bary"]
    fw = op["facet_w"][0] / op["facet_w"][0].sum()
    for row in rules:
        *pt, w = row
        pt = np.array(pt)
        hits = [j for j in range(len(fb)) if np.allclose(np.sort(fb[j]), np.sort(pt), atol=1e-12, rtol=0)]
        assert hits, pt
        for j in hits:
            assert abs(fw[j] - w) < 1e-12


def test_node_counts():
    counts = {(d, p): reference_operator(d, p)["n_p"] for d, p in CASES}
    assert counts == {(2, 1): 6, (2, 2): 10, (2, 3): 18, (2, 4): 22,
                      (3, 1): 12, (3, 2): 25, (3, 3): 60}
