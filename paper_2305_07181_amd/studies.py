"""Studies of the paper run through the library (MI355X).

    python -m paper_2305_07181_amd.studies conservation [--ns 60 80 100 120]
        [--ps 1 2 3 4] [--tf 2.0] [--cfl 0.1]
    python -m paper_2305_07181_amd.studies mms --dim 2|3 [--ns 6 9 12 15]
        [--ps 1 2 3] [--tf 0.001] [--steps 1000] [--mu 0.01] [--euler]
    python -m paper_2305_07181_amd.studies vortex2d [--ns 60 80 100 120]
        [--ps 1 2 3 4] [--tf 2.0] [--cfl 0.1] [--hadamard]
    python -m paper_2305_07181_amd.studies vortex3d [--ns 15 20 25 30]
        [--ps 1 2 3] [--tf 1.0] [--cfl 0.25]
    python -m paper_2305_07181_amd.studies tgv [--ns 24] [--ps 3] [--steps 100]
        [--cfl 0.1] [--re 1600] [--fp64]

Primary conservation (Sec. 4.3, Thm. conservation; the grid study of Sec. 7.3,
Table conservation): the 2D isentropic vortex of the paper's studies on its
curved grid sequence (n x n rectangles of [0,20] x [-5,5] cut into 2 n^2
triangles) is advanced by relaxation RK4 at the given CFL to t_f, and the
mass and energy errors

    |sum_k 1^T H_k u_k (t_f) - sum_k 1^T H_k u_k (0)| / |sum_k 1^T H_k u_k (0)|

are reported with their rates between consecutive grids (the run stops at
the first step that reaches t_f; its time is reported).

Manufactured solution (Sec. 7, the grid study of the manufactured solution
for the compressible Navier-Stokes equations, Table nse accuracy): the
fields rho = 2 + 0.1 sin(pi (sum_i x_i - 0.6 t)), V_i = 1 on [-1,1]^d start
from their nodal values and are advanced with the source (sbp_set_source)
by `steps` relaxation RK4 steps of dt = t_f / steps; the L2 error
of the paper's accuracy section (Sec. 7.3: the nodal solution interpolated
to a quadrature of degree 3p + 1, the squared error integrated and summed
over the elements and components, sbp_source_error with the quadrature
norm) and the nodal H-norm error sqrt(sum_c sum_k (u - u*)_c^T H_k
(u - u*)_c) at the final time are reported with their rates.  The
equations are the Navier-Stokes equations (mu, Pr = 0.71, R = 1, heat flux
on, Baumann-Oden SATs, no interface dissipation; --euler: the Euler
equations) on the study's curved grids: triangles and tetrahedra with
quadratic maps (in 3D at p = 1 the map moves the vertices of affine
tetrahedra, the map degree Assumption 1 allows).

2D isentropic vortex (Sec. 7.3, Table accuracy vortex 2d): the vortex of
sbp_set_source(SOURCE_VORTEX2D) on the curved grids n^2 x 2 of the
conservation study, conservative and dissipative SATs, relaxation RK4 at
CFL 0.1 until the first step at or past t_f = 2, the error in the paper's
norm at the time reached.

3D isentropic vortex (Sec. 7.3, Table accuracy vortex 3d): the vortex of
sbp_set_source(SOURCE_VORTEX3D) on the paper's curved grids n^3 x 6 of
[-10,10]^3 (quadratic maps for p >= 2, perturbed vertices of affine
tetrahedra for p = 1), entropy conservative and with matrix dissipation,
relaxation RK4 at CFL 0.25 until the first step at or past t_f = 1; the
error in the paper's norm at the time reached, with rates.

Viscous Taylor-Green vortex (Sec. 7.5): the history of the scaled kinetic
energy and of the total entropy over a number of relaxation RK4 steps on
n^3 x 6 tetrahedra (the paper compares the dissipation rate with reference
DNS data, which is not reproduced here).

Every step and every sum runs in the library (sbp_rrk_step,
sbp_diagnostics, sbp_source_state, sbp_source_error); this module only
builds the inputs and prints one JSON line per grid.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def conservation_run(n: int, p: int, tf: float = 2.0, cfl: float = 0.1) -> dict:
    import torch
    from . import sbp, workloads as wl
    desc = wl.paper_vortex2d_mesh(n)
    mesh = sbp.Mesh(desc, p)
    x = mesh.node_coords().cpu().numpy().reshape(mesh.n_elem, 2, -1)
    rho, V, pr = wl.paper_vortex2d(np.moveaxis(x, 1, 0))
    u = torch.from_numpy(np.ascontiguousarray(np.moveaxis(wl.conservative(rho, V, pr), 0, 1))).cuda()
    d0 = mesh.diagnostics(u)
    t, steps, t0 = 0.0, 0, time.perf_counter()
    while t < tf:   # time step from the CFL rule at every step (Sec. 7.1); the last may pass t_f
        rep = mesh.rrk_step(u, cfl=cfl)
        t = rep["t"]
        steps += 1
    d1 = mesh.diagnostics(u)
    mesh.check_device()
    nc = mesh.n_c
    out = dict(n=n, p=p, n_elem=int(mesh.n_elem), steps=steps, t=t, seconds=time.perf_counter() - t0,
               mass_error=abs(d1[1] - d0[1]) / abs(d0[1]),
               energy_error=abs(d1[nc] - d0[nc]) / abs(d0[nc]),
               entropy_change=(d1[0] - d0[0]) / abs(d0[0]))
    mesh.close()
    return out


def conservation_study(ns, ps, tf=2.0, cfl=0.1, emit=print):
    rows = []
    for p in ps:
        prev = None
        for n in ns:
            r = conservation_run(n, p, tf, cfl)
            if prev is not None:
                f = math.log(n / prev["n"])
                for k in ("mass", "energy"):
                    r[f"{k}_rate"] = math.log(prev[f"{k}_error"] / r[f"{k}_error"]) / f
            emit(json.dumps(r))
            rows.append(r)
            prev = r
    return rows


def mms_run(dim: int, n: int, p: int, tf: float = 1e-3, steps: int = 1000, mu: float = 0.01,
            viscous: bool = True) -> dict:
    from . import sbp, workloads as wl
    # the study's curved grids; in 3D at p = 1 the curving map moves the
    # vertices of affine tetrahedra (the map degree Assumption 1 allows there)
    desc = wl.mms_mesh2d(n) if dim == 2 else wl.mms_mesh3d(n, curve="quadratic" if p >= 2 else "vertices")
    mesh = sbp.Mesh(desc, p, viscous=viscous, mu=mu if viscous else 0.0, Pr=0.71, R=1.0)
    mesh.set_source()
    mesh.set_time(0.0)
    u = mesh.source_state(0.0)
    e0 = mesh.source_error(u, 0.0, "nodal")
    dt = tf / steps
    t0 = time.perf_counter()
    rep = None
    for _ in range(steps):
        rep = mesh.rrk_step(u, dt=dt)
    secs = time.perf_counter() - t0
    e = mesh.source_error(u, rep["t"], "quadrature")
    en = mesh.source_error(u, rep["t"], "nodal")
    mesh.check_device()
    out = dict(dim=dim, n=n, p=p, n_elem=int(mesh.n_elem), equations="navier-stokes" if viscous else "euler",
               steps=steps, t=rep["t"], seconds=secs,
               l2_error=math.sqrt(float(e.sum())), l2_error_rho=math.sqrt(float(e[0])),
               l2_error_nodal=math.sqrt(float(en.sum())), initial_error_nodal=math.sqrt(float(e0.sum())))
    mesh.close()
    return out


def mms_study(dim, ns, ps, tf=1e-3, steps=1000, mu=0.01, emit=print, viscous=True):
    rows = []
    for p in ps:
        prev = None
        for n in ns:
            r = mms_run(dim, n, p, tf, steps, mu, viscous)
            if prev is not None:
                f = math.log(n / prev["n"])   # h = (volume / n_e)^(1/d) falls as 1/n
                r["rate"] = math.log(prev["l2_error"] / r["l2_error"]) / f
                r["rate_nodal"] = math.log(prev["l2_error_nodal"] / r["l2_error_nodal"]) / f
            emit(json.dumps(r))
            rows.append(r)
            prev = r
    return rows


def vortex_run(dim: int, n: int, p: int, dissipation: bool, tf: float, cfl: float, hadamard: bool = False) -> dict:
    from . import sbp, workloads as wl
    if dim == 2:
        desc = wl.paper_vortex2d_mesh(n)
    else:
        desc = wl.paper_vortex3d_mesh(n, quadratic=p >= 2)
    mesh = sbp.Mesh(desc, p, dissipation=dissipation, form=sbp.FORM_HADAMARD if hadamard else sbp.FORM_SPLIT)
    mesh.set_source(sbp.SOURCE_VORTEX2D if dim == 2 else sbp.SOURCE_VORTEX3D)
    mesh.set_time(0.0)
    u = mesh.source_state(0.0)
    d0 = mesh.diagnostics(u)
    t, steps, t0 = 0.0, 0, time.perf_counter()
    while t < tf:
        t = mesh.rrk_step(u, cfl=cfl)["t"]
        steps += 1
    secs = time.perf_counter() - t0
    e = mesh.source_error(u, t, "quadrature")
    d1 = mesh.diagnostics(u)
    mesh.check_device()
    out = dict(dim=dim, n=n, p=p, n_elem=int(mesh.n_elem), form="hadamard" if hadamard else "split",
               dissipation=dissipation, steps=steps, t=t,
               seconds=secs, l2_error=math.sqrt(float(e.sum())), entropy_change=(d1[0] - d0[0]) / abs(d0[0]))
    mesh.close()
    return out


def vortex3d_run(n: int, p: int, dissipation: bool, tf: float = 1.0, cfl: float = 0.25) -> dict:
    return vortex_run(3, n, p, dissipation, tf, cfl)


def vortex_study(dim, ns, ps, tf, cfl, emit=print, hadamard=False):
    rows = []
    for p in ps:
        for diss in (False, True):
            prev = None
            for n in ns:
                r = vortex_run(dim, n, p, diss, tf, cfl, hadamard)
                if prev is not None:   # h = (volume / n_e)^(1/d) falls as 1/n
                    r["rate"] = math.log(prev["l2_error"] / r["l2_error"]) / math.log(n / prev["n"])
                emit(json.dumps(r))
                rows.append(r)
                prev = r
    return rows


def tgv_run(n: int = 24, p: int = 3, steps: int = 100, re: float = 1600.0, cfl: float = 0.1,
            precision: str = "fp32", emit=None) -> dict:
    """Viscous Taylor-Green vortex (Sec. 7.5) on n^3 x 6 tetrahedra of
    [0, 2 pi]^3, M = 0.1, Pr = 0.71, mu = 1 / Re, heat flux and matrix
    dissipation on, relaxation RK4 (captured stage graph) at the given CFL:
    the scaled kinetic energy E_k = sum H rho |V|^2 / 2 / (rho_0 |Omega|) and
    the total entropy after every step, and the dissipation rate
    epsilon = -dE_k/dt from second-order differences of the history on its
    (variable) time points."""
    import torch
    from . import sbp, workloads as wl
    desc = wl.tgv_mesh(n)
    mesh = sbp.Mesh(desc, p, precision=sbp.FP32 if precision == "fp32" else sbp.FP64, dissipation=True,
                    viscous=True, heat_flux=True, mu=1.0 / re, Pr=0.71, R=1.0)
    x = mesh.node_coords().cpu().numpy().reshape(mesh.n_elem, 3, -1)
    rho, V, pr = wl.taylor_green(np.moveaxis(x, 1, 0))
    u = torch.from_numpy(np.ascontiguousarray(np.moveaxis(wl.conservative(rho, V, pr), 0, 1))).cuda()
    vol = (2.0 * math.pi) ** 3
    nc = mesh.n_c
    d = mesh.diagnostics(u)
    ts, eks, ss, gammas = [0.0], [d[nc + 1] / vol], [d[0]], []
    t0 = time.perf_counter()
    for k in range(steps):
        rep = mesh.rrk_step(u, cfl=cfl)
        d = mesh.diagnostics(u)
        ts.append(rep["t"])
        eks.append(d[nc + 1] / vol)
        ss.append(d[0])
        gammas.append(rep["gamma"])
        if emit is not None and (k + 1) % 10 == 0:
            emit(json.dumps(dict(step=k + 1, t=ts[-1], E_k=eks[-1], entropy=ss[-1], gamma=rep["gamma"])))
    secs = time.perf_counter() - t0
    mesh.check_device()
    mesh.close()
    t, ek = np.array(ts), np.array(eks)
    eps = -np.gradient(ek, t)      # second order on non-uniform points, one-sided at the ends
    return dict(n=n, p=p, n_elem=6 * n ** 3, precision=precision, re=re, cfl=cfl, steps=steps, seconds=secs,
                t=ts, E_k=eks, entropy=ss, epsilon=eps.tolist(), gamma_min=min(gammas), gamma_max=max(gammas))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["conservation", "mms", "vortex2d", "vortex3d", "tgv"])
    ap.add_argument("--ns", type=int, nargs="+")
    ap.add_argument("--ps", type=int, nargs="+")
    ap.add_argument("--tf", type=float)
    ap.add_argument("--cfl", type=float, default=0.1)
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--mu", type=float, default=0.01)
    ap.add_argument("--hadamard", action="store_true", help="vortex studies: the Hadamard form (comparator)")
    ap.add_argument("--re", type=float, default=1600.0, help="tgv: Reynolds number")
    ap.add_argument("--fp64", action="store_true", help="tgv: FP64 residuals (default FP32)")
    ap.add_argument("--euler", action="store_true", help="mms: the Euler equations (no viscous terms)")
    a = ap.parse_args(argv)
    emit = lambda s: print(s, flush=True)
    if a.study == "conservation":
        conservation_study(a.ns or [60, 80, 100, 120], a.ps or [1, 2, 3, 4], a.tf or 2.0, a.cfl, emit=emit)
    elif a.study == "vortex3d":
        vortex_study(3, a.ns or [15, 20, 25, 30], a.ps or [1, 2, 3], a.tf or 1.0, a.cfl if a.cfl != 0.1 else 0.25,
                     emit=emit, hadamard=a.hadamard)
    elif a.study == "tgv":
        for n in a.ns or [24]:
            for p in a.ps or [3]:
                r = tgv_run(n, p, a.steps if a.steps != 1000 else 100, a.re, a.cfl,
                            "fp64" if a.fp64 else "fp32", emit=emit)
                emit(json.dumps(r))
    elif a.study == "vortex2d":
        vortex_study(2, a.ns or [60, 80, 100, 120], a.ps or [1, 2, 3, 4], a.tf or 2.0, a.cfl, emit=emit,
                     hadamard=a.hadamard)
    else:
        ns = a.ns or ([20, 30, 40, 50] if a.dim == 2 else [6, 9, 12, 15])
        ps = a.ps or ([1, 2, 3, 4] if a.dim == 2 else [1, 2, 3])
        mms_study(a.dim, ns, ps, a.tf or 1e-3, a.steps, a.mu, emit=emit, viscous=not a.euler)


if __name__ == "__main__":
    sys.exit(main())
