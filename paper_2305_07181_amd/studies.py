"""Studies of the paper run through the library (MI355X).

    python -m paper_2305_07181_amd.studies conservation [--ns 60 80 100 120]
        [--ps 1 2 3 4] [--tf 2.0] [--cfl 0.1]

Primary conservation (Sec. 4.3, Thm. conservation; the grid study of Sec. 7.3,
Table conservation): the 2D isentropic vortex of the paper's studies on its
curved grid sequence (n x n rectangles of [0,20] x [-5,5] cut into 2 n^2
triangles) is advanced by relaxation RK4 at the given CFL to t_f, and the
mass and energy errors

    |sum_k 1^T H_k u_k (t_f) - sum_k 1^T H_k u_k (0)| / |sum_k 1^T H_k u_k (0)|

are reported with their rates between consecutive grids (the run stops at
the first step that reaches t_f; its time is reported).  Every step and
every sum runs in the library (sbp_rrk_step, sbp_diagnostics); this module
only builds the inputs and prints one JSON line per grid.
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["conservation"])
    ap.add_argument("--ns", type=int, nargs="+", default=[60, 80, 100, 120])
    ap.add_argument("--ps", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--tf", type=float, default=2.0)
    ap.add_argument("--cfl", type=float, default=0.1)
    a = ap.parse_args(argv)
    conservation_study(a.ns, a.ps, a.tf, a.cfl, emit=lambda s: print(s, flush=True))


if __name__ == "__main__":
    sys.exit(main())
