"""Seeded synthetic inputs: periodic meshes and initial states.

This module is the only code shared by the HIP path's tests/benchmarks and the
CPU oracle.  It holds no arithmetic of the discretization itself: it builds
mesh descriptions (vertex coordinates, connectivity, quadratic geometry nodes)
and evaluates analytic initial conditions at coordinates supplied by the
caller.  Every random draw comes from ``numpy.random.default_rng(seed)`` with
the seed stated at the call site.

Workloads (shapes follow the paper's test problems, Sec. 7):
  * periodic square split into right triangles (Sec. 7.3 accuracy meshes);
  * periodic cube split into six tetrahedra per hexahedron (Sec. 7.3 and 7.5);
  * optional quadratic (P2) warp of the triangle mesh (curved meshes, Sec. 7.3);
  * isentropic vortex, Taylor-Green vortex and smooth random Fourier states.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GAMMA = 1.4

# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------


def periodic_tri_mesh(nx: int, ny: int, lx: float, ly: float | None = None,
                      warp: float = 0.0) -> dict:
    """Periodic [0,lx]x[0,ly] grid of nx*ny quads, each cut along its
    (i,j)->(i+1,j+1) diagonal into two positively oriented triangles.

    Boundary vertices are duplicated (the x=lx column is distinct from x=0);
    periodicity is expressed by ``period`` and recovered by coordinate
    matching.  With ``warp`` != 0 the quadratic geometry nodes (vertices and
    edge midpoints) are displaced by
        delta = warp * L * sin(2 pi x/L) sin(2 pi y/L)
    added to both coordinates (L = lx = ly), which vanishes on the box edges
    so the curved mesh stays conforming and periodic.

    Returns a mesh description dict:
      dim=2, vert_xyz[n_vert,2], elem_vert[n_elem,3], period[2],
      p_geom (1 or 2), geom_nodes[n_elem,6,2] (P2 node order: v0, v1, v2,
      mid(v0,v1), mid(v1,v2), mid(v2,v0)) or None.
    """
    ly = lx if ly is None else ly
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    vert = np.stack([X.ravel(), Y.ravel()], 1)

    def vid(i, j):
        return i * (ny + 1) + j

    elems = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            elems.append((a, b, c))
            elems.append((a, c, d))
    elem = np.array(elems, dtype=np.int32)
    desc = dict(dim=2, vert_xyz=vert, elem_vert=elem,
                period=np.array([lx, ly], dtype=np.float64), p_geom=1,
                geom_nodes=None)
    if warp != 0.0:
        if abs(lx - ly) > 0:
            raise ValueError("warp needs a square box")
        L = lx
        v = vert[elem]                                   # [ne,3,2]
        mids = np.stack([0.5 * (v[:, 0] + v[:, 1]), 0.5 * (v[:, 1] + v[:, 2]),
                         0.5 * (v[:, 2] + v[:, 0])], 1)
        g = np.concatenate([v, mids], 1)                  # [ne,6,2]
        dlt = warp * L * np.sin(2 * np.pi * g[..., 0] / L) * np.sin(2 * np.pi * g[..., 1] / L)
        g = g + dlt[..., None]
        desc["p_geom"] = 2
        desc["geom_nodes"] = np.ascontiguousarray(g)
    return desc


# The six tetrahedra of the Kuhn (Freudenthal) split of the unit cube: the
# path 0 -> e_s1 -> e_s1+e_s2 -> (1,1,1) for every permutation s.  The split
# is translation invariant, hence conforming across cubes and periodic.
_KUHN = []
for _s in itertools.permutations(range(3)):
    _p = [np.zeros(3, dtype=int)]
    for _k in _s:
        _q = _p[-1].copy()
        _q[_k] = 1
        _p.append(_q)
    _KUHN.append(_p)


def periodic_tet_mesh(n: int, L: float) -> dict:
    """Periodic [0,L]^3 grid of n^3 hexahedra, each split into six
    positively oriented tetrahedra (Kuhn split).  Boundary vertices are
    duplicated as in :func:`periodic_tri_mesh`."""
    g = np.linspace(0.0, L, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    vert = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)

    def vid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    elems = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for path in _KUHN:
                    ids = [vid(i + q[0], j + q[1], k + q[2]) for q in path]
                    x = vert[ids]
                    vol = np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], 1))
                    if vol < 0:
                        ids[1], ids[2] = ids[2], ids[1]
                    elems.append(ids)
    elem = np.array(elems, dtype=np.int32)
    return dict(dim=3, vert_xyz=vert, elem_vert=elem,
                period=np.array([L, L, L], dtype=np.float64), p_geom=1,
                geom_nodes=None)


# ----------------------------------------------------------------------------
# states (primitive variables rho, V, p at given coordinates)
# ----------------------------------------------------------------------------


def conservative(rho, V, p, gamma=GAMMA):
    """Stack primitive fields into the conservative vector of the governing
    equations (Sec. 2.2): [rho, rho V, p/(gamma-1) + rho |V|^2 / 2].
    Shapes: rho,p [...], V [d,...] -> [d+2,...]."""
    rho = np.asarray(rho, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    e = p / (gamma - 1.0) + 0.5 * rho * np.sum(V * V, axis=0)
    return np.concatenate([rho[None], rho[None] * V, np.asarray(e)[None]], 0)


def isentropic_vortex(x, t=0.0, eps=5.0, center=(10.0, 10.0), vinf=(1.0, 1.0),
                      period=(20.0, 20.0), gamma=GAMMA):
    """Standard isentropic vortex advected by the free stream ``vinf`` on a
    periodic box (minimum-image distance to the moving centre).

    x: [2, ...] coordinates.  Returns (rho, V[2,...], p) with rho_inf = p_inf = 1.
        T = 1 - (gamma-1) eps^2/(8 gamma pi^2) exp(1 - r^2),
        (u,v) = vinf + eps/(2 pi) exp((1-r^2)/2) (-(y-yc), x-xc),
        rho = T^(1/(gamma-1)), p = rho^gamma.
    """
    x = np.asarray(x, dtype=np.float64)
    dx = x[0] - (center[0] + vinf[0] * t)
    dy = x[1] - (center[1] + vinf[1] * t)
    dx = dx - period[0] * np.round(dx / period[0])
    dy = dy - period[1] * np.round(dy / period[1])
    r2 = dx * dx + dy * dy
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    f = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    V = np.stack([vinf[0] - f * dy, vinf[1] + f * dx], 0)
    return rho, V, p


def taylor_green(x, mach=0.1, gamma=GAMMA):
    """Taylor-Green vortex initial condition (Sec. 7.5) with u0 = rho0 = R = L = 1,
    p0 = 1/(gamma M^2), T0 = p0, on coordinates x [3,...] (the initial field is
    2 pi periodic, so [0, 2 pi]^3 is a shift of the paper's [-pi, pi]^3)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = 1.0 / (gamma * mach * mach)
    T0 = p0
    u = np.sin(x[0]) * np.cos(x[1]) * np.cos(x[2])
    v = -np.cos(x[0]) * np.sin(x[1]) * np.cos(x[2])
    w = np.zeros_like(u)
    p = p0 + (1.0 / 16.0) * (np.cos(2 * x[0]) + np.cos(2 * x[1])) * (np.cos(2 * x[2]) + 2.0)
    rho = p / T0
    return rho, np.stack([u, v, w], 0), p


def fourier_modes(seed: int, dim: int, K: int, n_modes: int = 8):
    """Draw the parameters of one smooth periodic field
        g(x) = sum_m a_m cos(2 pi k_m . x / L + phi_m),  sum a_m = 1,
    with a_m ~ U(0,1) normalised, k_m in {-K..K}^dim \\ {0}, phi_m ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, n_modes)
    a = a / a.sum()
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-K, K + 1, dim)
        if np.any(k != 0):
            ks.append(k)
    phi = rng.uniform(0.0, 2 * math.pi, n_modes)
    return a, np.array(ks, dtype=np.float64), phi


def fourier_field(x, modes, L):
    a, ks, phi = modes
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros(x.shape[1:])
    for am, km, pm in zip(a, ks, phi):
        arg = 2 * math.pi * np.tensordot(km, x, axes=(0, 0)) / L + pm
        g = g + am * np.cos(arg)
    return g


def random_smooth_state(x, seed: int, L: float, K: int = 3, amp: float = 0.5,
                        vamp: float = 0.5):
    """Smooth random periodic state: rho = 1 + amp g_rho, p = 1 + amp g_p,
    V_i = vamp/sqrt(d) g_{V_i}; each g from an independent seeded Fourier
    draw (|g| <= 1), so rho, p in [1-amp, 1+amp] and |V| <= vamp."""
    x = np.asarray(x, dtype=np.float64)
    dim = x.shape[0]
    ss = np.random.SeedSequence(seed).spawn(dim + 2)
    seeds = [int(s.generate_state(1)[0]) for s in ss]
    g = [fourier_field(x, fourier_modes(s, dim, K), L) for s in seeds]
    rho = 1.0 + amp * g[0]
    p = 1.0 + amp * g[1]
    V = np.stack([vamp / math.sqrt(dim) * g[2 + i] for i in range(dim)], 0)
    return rho, V, p


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------


def vortex2d_mesh(n: int = 8, warp: float = 0.0) -> dict:
    """[0,20]^2, n x n quads -> 2 n^2 triangles (n=8: the 128-triangle case;
    n=128 with warp 0.05: the 32768-triangle curved case)."""
    return periodic_tri_mesh(n, n, 20.0, 20.0, warp=warp)


def paper_vortex2d_mesh(n: int) -> dict:
    """Grid of the paper's 2D isentropic-vortex studies (Sec. 7.3): the
    periodic box [0,20] x [-5,5] in n x n rectangles, each cut into two
    triangles, with the quadratic geometry nodes (vertices and edge midpoints)
    moved by the perturbation of eq. (curve 2d vortex),
        x1 = x1^ + 1/8 cos(pi/20 (x1^ - 10)) cos(3 pi/10 x2^),
        x2 = x2^ + 1/8 sin(pi/5 (x1 - 10)) cos(pi/10 x2^)   (x1 perturbed),
    which vanishes on the box edges (conforming and periodic)."""
    desc = periodic_tri_mesh(n, n, 20.0, 10.0)
    vert = desc["vert_xyz"].copy()
    vert[:, 1] -= 5.0
    v = vert[desc["elem_vert"]]                            # [ne,3,2]
    mids = np.stack([0.5 * (v[:, 0] + v[:, 1]), 0.5 * (v[:, 1] + v[:, 2]),
                     0.5 * (v[:, 2] + v[:, 0])], 1)
    g = np.concatenate([v, mids], 1)                       # [ne,6,2]
    x1 = g[..., 0] + 0.125 * np.cos(np.pi / 20 * (g[..., 0] - 10)) * np.cos(0.3 * np.pi * g[..., 1])
    x2 = g[..., 1] + 0.125 * np.sin(np.pi / 5 * (x1 - 10)) * np.cos(np.pi / 10 * g[..., 1])
    desc["vert_xyz"] = vert
    desc["p_geom"] = 2
    desc["geom_nodes"] = np.ascontiguousarray(np.stack([x1, x2], -1))
    return desc


def paper_vortex2d(x, t=0.0, alpha=3.0, center=(5.0, 0.0), period=(20.0, 10.0), gamma=GAMMA):
    """The 2D isentropic vortex of the paper's studies (Sec. 7.3): strength
    alpha = 3, centre (5, 0) advected by the free stream (1, 0) on the periodic
    box [0,20] x [-5,5] (minimum-image distance), velocity perturbation
    alpha/(2 pi) exp(1 - r^2) (-(y - yc), x - xc) and, for radial
    equilibrium, T = 1 - alpha^2 (gamma-1) / (16 gamma pi^2) exp(2 (1 - r^2)),
    rho = T^(1/(gamma-1)), p = rho^gamma.  Returns (rho, V[2,...], p)."""
    x = np.asarray(x, dtype=np.float64)
    dx = x[0] - (center[0] + t)
    dy = x[1] - center[1]
    dx = dx - period[0] * np.round(dx / period[0])
    dy = dy - period[1] * np.round(dy / period[1])
    r2 = dx * dx + dy * dy
    T = 1.0 - alpha * alpha * (gamma - 1.0) / (16.0 * gamma * math.pi ** 2) * np.exp(2.0 * (1.0 - r2))
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    f = alpha / (2.0 * math.pi) * np.exp(1.0 - r2)
    V = np.stack([1.0 - f * dy, f * dx], 0)
    return rho, V, p


def mms_mesh2d(n: int) -> dict:
    """Grid of the paper's manufactured-solution study (Sec. 7): the periodic
    box [-1,1]^2 in n x n squares, each cut into two triangles, with the
    quadratic geometry nodes moved by the curving map of that study,
        x_i = x^_i + 1/8 cos(pi/2 x^_i) prod_{j != i} sin(pi x^_j),
    which fixes every point of the box edges (conforming and periodic)."""
    desc = periodic_tri_mesh(n, n, 2.0, 2.0)
    vert = desc["vert_xyz"] - 1.0
    v = vert[desc["elem_vert"]]                            # [ne,3,2]
    mids = np.stack([0.5 * (v[:, 0] + v[:, 1]), 0.5 * (v[:, 1] + v[:, 2]),
                     0.5 * (v[:, 2] + v[:, 0])], 1)
    g = np.concatenate([v, mids], 1)                       # [ne,6,2]
    x1 = g[..., 0] + 0.125 * np.cos(0.5 * np.pi * g[..., 0]) * np.sin(np.pi * g[..., 1])
    x2 = g[..., 1] + 0.125 * np.cos(0.5 * np.pi * g[..., 1]) * np.sin(np.pi * g[..., 0])
    desc["vert_xyz"] = vert
    desc["p_geom"] = 2
    desc["geom_nodes"] = np.ascontiguousarray(np.stack([x1, x2], -1))
    return desc


def mms_mesh3d(n: int, curve: str = "none") -> dict:
    """The periodic box [-1,1]^3 of the manufactured-solution study in n^3
    cubes of six tetrahedra each.  curve: "none" (affine tetrahedra),
    "quadratic" (the study's curving map
        x_i = x^_i + 1/8 cos(pi/2 x^_i) prod_{j != i} sin(pi x^_j)
    applied to the quadratic map nodes, vertices and edge midpoints; degrees
    p >= 2) or "vertices" (the map applied to the vertices of affine
    tetrahedra, the map degree Assumption 1 allows at p = 1).  The map fixes
    every point of the box faces (conforming and periodic)."""
    desc = periodic_tet_mesh(n, 2.0)
    desc["vert_xyz"] = desc["vert_xyz"] - 1.0

    def curved(x):
        s = np.sin(np.pi * x)
        c = np.cos(0.5 * np.pi * x)
        return np.stack([x[..., 0] + 0.125 * c[..., 0] * s[..., 1] * s[..., 2],
                         x[..., 1] + 0.125 * c[..., 1] * s[..., 0] * s[..., 2],
                         x[..., 2] + 0.125 * c[..., 2] * s[..., 0] * s[..., 1]], -1)

    if curve == "vertices":
        desc["vert_xyz"] = np.ascontiguousarray(curved(desc["vert_xyz"]))
    elif curve == "quadratic":
        desc["p_geom"] = 2
        desc["geom_nodes"] = np.ascontiguousarray(curved(_tet_p2_nodes(desc)))
    elif curve != "none":
        raise ValueError(curve)
    return desc


# Edge midpoints of the quadratic tetrahedron, in the order of its map nodes
# 4..9 (after the four vertices).
P2_TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def _tet_p2_nodes(desc):
    v = desc["vert_xyz"][desc["elem_vert"]]                  # [ne,4,3]
    mids = np.stack([0.5 * (v[:, a] + v[:, b]) for a, b in P2_TET_EDGES], 1)
    return np.concatenate([v, mids], 1)                      # [ne,10,3]


def curved_tet_mesh(n: int, L: float, warp: float) -> dict:
    """Periodic [0,L]^3 in n^3 cubes of six tetrahedra with quadratic maps:
    the map nodes (vertices and edge midpoints) are moved by
        delta = warp * L * sin(2 pi x/L) sin(2 pi y/L) sin(2 pi z/L)
    added to every coordinate, which vanishes on the box faces (conforming
    and periodic)."""
    desc = periodic_tet_mesh(n, L)
    g = _tet_p2_nodes(desc)
    s = np.sin(2 * np.pi * g / L)
    dlt = warp * L * s[..., 0] * s[..., 1] * s[..., 2]
    desc["p_geom"] = 2
    desc["geom_nodes"] = np.ascontiguousarray(g + dlt[..., None])
    return desc


def paper_vortex3d_mesh(n: int, quadratic: bool = True) -> dict:
    """Grid of the paper's 3D isentropic-vortex study (Sec. 7.3): the
    periodic box [-10,10]^3 in n^3 cubes of six tetrahedra, moved by
    x_i = x^_i + 0.05 sin(pi x^_i / 2) (eq. curve 3d vortex), which fixes the
    box faces: the quadratic map nodes (quadratic=True, degrees p >= 2), or
    only the vertices of affine tetrahedra (p = 1, the map degree Assumption
    1 allows there)."""
    desc = periodic_tet_mesh(n, 20.0)
    desc["vert_xyz"] = desc["vert_xyz"] - 10.0
    if not quadratic:
        v = desc["vert_xyz"]
        desc["vert_xyz"] = np.ascontiguousarray(v + 0.05 * np.sin(0.5 * np.pi * v))
        return desc
    g = _tet_p2_nodes(desc)
    desc["p_geom"] = 2
    desc["geom_nodes"] = np.ascontiguousarray(g + 0.05 * np.sin(0.5 * np.pi * g))
    return desc


def tgv_mesh(n: int) -> dict:
    """[0, 2 pi]^3, n^3 hexes x 6 tetrahedra (n=32: 196608; n=24: 82944)."""
    return periodic_tet_mesh(n, 2 * math.pi)


def batch_problem_specs(n_problems: int = 48, seed: int = 0):
    """Sizes of the batched 2D workload: per problem a degree p ~ U{1..4} and
    an element target n_e ~ logU[256, 16384], realised as an Nx x Ny periodic
    grid on [0,1]^2 with Nx = max(2, round(sqrt(n_e/2))),
    Ny = max(2, round(n_e/(2 Nx))), actual n_e = 2 Nx Ny."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_problems):
        p = int(rng.integers(1, 5))
        ne = float(np.exp(rng.uniform(math.log(256), math.log(16384))))
        nx = max(2, int(round(math.sqrt(ne / 2))))
        ny = max(2, int(round(ne / (2 * nx))))
        out.append(dict(p=p, nx=nx, ny=ny, seed=1000 + b))
    return out


def batch_mesh(specs, warp: float = 0.0):
    """The problems of ``batch_problem_specs`` as one mesh description: each
    an nx x ny periodic grid of triangles on [0,1]^2 with its own vertices.
    Returns (desc, degree[n_elem], problem_off[n_problems + 1])."""
    verts, elems, geoms, degs, off = [], [], [], [], [0]
    nv = 0
    for sp in specs:
        d = periodic_tri_mesh(sp["nx"], sp["ny"], 1.0, 1.0, warp)
        verts.append(d["vert_xyz"])
        elems.append(d["elem_vert"] + nv)
        nv += len(d["vert_xyz"])
        if warp != 0.0:
            geoms.append(d["geom_nodes"])
        degs.append(np.full(len(d["elem_vert"]), sp["p"], dtype=np.int32))
        off.append(off[-1] + len(d["elem_vert"]))
    desc = dict(dim=2, vert_xyz=np.concatenate(verts), elem_vert=np.concatenate(elems).astype(np.int32),
                period=np.array([1.0, 1.0]), p_geom=2 if warp != 0.0 else 1,
                geom_nodes=np.concatenate(geoms) if warp != 0.0 else None)
    return desc, np.concatenate(degs), np.array(off, dtype=np.int32)


def copies_mesh(desc: dict, degrees):
    """One mesh description of len(degrees) independent copies of a 2D mesh
    with quadratic maps (its own vertices per copy, the same period), copy b
    of degree degrees[b].  Returns (desc, degree[n_elem], problem_off[n + 1])
    as ``batch_mesh``."""
    verts, elems, geoms, degs, off = [], [], [], [], [0]
    nv = 0
    for p in degrees:
        verts.append(desc["vert_xyz"])
        elems.append(desc["elem_vert"] + nv)
        nv += len(desc["vert_xyz"])
        geoms.append(desc["geom_nodes"])
        degs.append(np.full(len(desc["elem_vert"]), p, dtype=np.int32))
        off.append(off[-1] + len(desc["elem_vert"]))
    out = dict(dim=2, vert_xyz=np.concatenate(verts), elem_vert=np.concatenate(elems).astype(np.int32),
               period=desc["period"], p_geom=2, geom_nodes=np.concatenate(geoms))
    return out, np.concatenate(degs), np.array(off, dtype=np.int32)


def sub_mesh(desc: dict, lo: int, hi: int) -> dict:
    """Elements [lo, hi) of a batched description as a mesh of their own."""
    ev = desc["elem_vert"][lo:hi]
    used = np.unique(ev)
    remap = np.full(len(desc["vert_xyz"]), -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    out = dict(desc)
    out["vert_xyz"] = desc["vert_xyz"][used]
    out["elem_vert"] = remap[ev].astype(np.int32)
    if desc.get("geom_nodes") is not None:
        out["geom_nodes"] = desc["geom_nodes"][lo:hi]
    return out
