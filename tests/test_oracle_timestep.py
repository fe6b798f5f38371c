"""Pins for the oracle's time-step rule (Sec. 7.1):

    dt = CFL * min_k h_min,k / |lambda|_max,k,

h_min,k the smallest distance between two SBP nodes of element k and
|lambda|_max,k the largest |V| + a over its nodes (a = sqrt(gamma p / rho)).

The expected values come from closed forms, not from the oracle's operators:
on triangles of degree p = 1, 2 the nodes nearest a vertex are the
Gauss-Legendre points of the edges (p + 1 points per edge, at the fraction
t_p of the edge from either end: t_1 = 1/2 - 1/(2 sqrt 3), t_2 = 1/2 -
sqrt(3/5)/2), and at degree 1 those are all the nodes.  On the grid of
a x a squares cut along one diagonal the closest pair sits at a 45-degree
corner, one node on a leg and one on the hypotenuse: h_min = t_p a.
A plausible slip in the rule fails one of these tests: dropping the sound
speed (the uniform state), the largest instead of the smallest node distance
(the uniform state), a mean over elements instead of the minimum (the
faster or smaller element), or a maximum over elements of h_min alone (the
refinement ratio and the moved vertex).
"""
import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle.geometry import OracleMesh
from oracle.residual import OracleScheme
from paper_2305_07181_amd import workloads as wl

T_GL = {1: 0.5 - 0.5 / math.sqrt(3.0), 2: 0.5 - 0.5 * math.sqrt(0.6)}
GAMMA = 1.4


def uniform_state(m, rho, V, p):
    x = m.node_coords()                       # [ne, 2, n_p]
    ne, _, n_p = x.shape
    R = np.full((ne, n_p), rho)
    Vx = np.full((ne, n_p), V[0])
    Vy = np.full((ne, n_p), V[1])
    P = np.full((ne, n_p), p)
    return np.moveaxis(wl.conservative(R, np.stack([Vx, Vy]), P), 0, 1).copy()


def speed(rho, V, p):
    return math.hypot(*V) + math.sqrt(GAMMA * p / rho)


@pytest.mark.parametrize("p", [1, 2])
def test_uniform_state_closed_form(p):
    n, L = 4, 20.0
    a = L / n
    m = OracleMesh(wl.periodic_tri_mesh(n, n, L), p)
    s = OracleScheme(m, ph.Gas())
    rho, V, pr = 1.2, (0.3, -0.4), 0.9
    u = uniform_state(m, rho, V, pr)
    cfl = 0.37
    expect = cfl * T_GL[p] * a / speed(rho, V, pr)
    assert abs(s.timestep(u, cfl) - expect) <= 1e-13 * expect


@pytest.mark.parametrize("p", [1, 2])
def test_time_step_scales_with_the_mesh_size(p):
    dts = []
    for n in (3, 6):
        m = OracleMesh(wl.periodic_tri_mesh(n, n, 12.0), p)
        s = OracleScheme(m, ph.Gas())
        dts.append(s.timestep(uniform_state(m, 1.0, (0.5, 0.0), 1.0), 0.1))
    assert abs(dts[0] / dts[1] - 2.0) <= 1e-13


def test_fastest_element_decides():
    """One element carries a faster flow: dt comes from that element alone."""
    n, L = 4, 20.0
    a = L / n
    m = OracleMesh(wl.periodic_tri_mesh(n, n, L), 1)
    s = OracleScheme(m, ph.Gas())
    u = uniform_state(m, 1.0, (0.2, 0.1), 1.0)
    fast = uniform_state(m, 0.8, (1.3, -0.6), 1.1)
    e_star = 9
    u[e_star] = fast[e_star]
    expect = 0.1 * T_GL[1] * a / speed(0.8, (1.3, -0.6), 1.1)
    assert abs(s.timestep(u, 0.1) - expect) <= 1e-13 * expect


def test_moved_vertex_smallest_element_decides():
    """An interior vertex is moved: the six triangles around it change shape;
    h_min of every element is recomputed here by brute force over its six
    degree-1 nodes (the two Gauss-Legendre points of each edge) and dt is the
    CFL times the smallest h_min over the flow speed."""
    n, L = 4, 20.0
    desc = wl.periodic_tri_mesh(n, n, L)
    vert = desc["vert_xyz"].copy()
    vid = 2 * (n + 1) + 2                      # vertex (i, j) = (2, 2)
    vert[vid] += np.array([0.31, -0.12]) * (L / n)
    desc = dict(desc, vert_xyz=vert)
    m = OracleMesh(desc, 1)
    s = OracleScheme(m, ph.Gas())
    rho, V, pr = 1.0, (0.25, 0.5), 1.3
    u = uniform_state(m, rho, V, pr)
    t = T_GL[1]
    hmins = []
    for ev in desc["elem_vert"]:
        x = vert[ev]
        pts = []
        for q in range(3):
            A, B = x[q], x[(q + 1) % 3]
            pts += [A + t * (B - A), B + t * (A - B)]
        pts = np.array(pts)
        d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
        hmins.append(d[np.triu_indices(6, 1)].min())
    hmins = np.array(hmins)
    assert hmins.min() < 0.95 * t * L / n      # the moved vertex made a smaller element
    expect = 0.2 * hmins.min() / speed(rho, V, pr)
    assert abs(s.timestep(u, 0.2) - expect) <= 1e-13 * expect
