"""Benchmark: residual elem-DOF updates/s of the entropy-split SBP residual on
one MI355X (FP64 vs FP32 vs the Hadamard form; VJP/forward time), with a
roofline object for every timed kernel family and the CPU oracle as a
reported baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One timed step = one FP64 entropy-split residual evaluation for each degree
p = 1..4 on the curved periodic 128x128x2 = 32768-triangle mesh (isentropic
vortex state, inputs resident in HBM), the four in one batched launch (one
mesh holding four independent copies of the grid, one per degree).  value =
sum_p n_elem n_p(p) / step time.  The breakdown gives, per family (2D, 3D affine and curved
tetrahedra, Navier-Stokes, the 48-problem batch), the FP64 and FP32 entropy
split, the Hadamard form and the VJP, each with its launch time and roofline
(algorithmic flops and bytes per element, the bound, the fraction of peak,
and HBM bytes from counter runs where they were taken on the same kernel
sources); the FP32 error against the FP64 residual per configuration; a
state with interface jumps; RRK4 steps (captured graph and eager); and the
CPU oracle on all host cores and on one.

    python bench.py --probe-kernels FILE

runs every timed call once per kernel variant between two marker kernels
(for HBM byte counter runs under rocprofv3) and writes the call list to FILE.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "residual elem-DOF updates/s: FP64 vs FP32 vs Hadamard form; VJP/forward time"
PEAK_HBM = 8.0e12          # B/s
PEAK_F64 = 78.6e12         # FLOP/s (vector and MFMA)
PEAK_F32 = 157.3e12        # FLOP/s (vector and dense MFMA)

# HBM bytes per call (FETCH_SIZE and WRITE_SIZE counter runs of
# `bench.py --probe-kernels`, calibrated against a plain device copy; see
# profiles/hbm_bytes_all_families.md), keyed "<row>/<name>/v<variant>".
# Valid only for the kernel sources they were taken on (TRAFFIC_SHA).
TRAFFIC_SHA = "3af9f721533f8a49"
TRAFFIC = {
    "batch48/fwd/v0": 1.999e+08,
    "batch48/vjp/v0": 5.152e+08,
    "jitter_p1/fp64_split/v0": 2.56e+07,
    "jitter_p1/fp64_split/v1": 1.731e+07,
    "jitter_p1/fp64_split/v2": 2.581e+07,
    "jitter_p2/fp64_split/v0": 2.654e+07,
    "jitter_p2/fp64_split/v1": 2.638e+07,
    "jitter_p2/fp64_split/v2": 2.676e+07,
    "jitter_p3/fp64_split/v0": 4.416e+07,
    "jitter_p3/fp64_split/v1": 4.398e+07,
    "jitter_p3/fp64_split/v2": 4.448e+07,
    "jitter_p4/fp64_split/v0": 5.323e+07,
    "jitter_p4/fp64_split/v1": 5.305e+07,
    "jitter_p4/fp64_split/v2": 5.396e+07,
    "ns_tgv_82944_p3/fp32_residual/v0": 7.99e+08,
    "ns_tgv_82944_p3/fp64_residual/v0": 1.23e+09,
    "ns_tgv_82944_p3/fp64_vjp/v0": 5.228e+09,
    "tet_p2_tgv_196608/fp32_split/v0": 6.686e+08,
    "tet_p2_tgv_196608/fp32_split/v1": 6.979e+08,
    "tet_p2_tgv_196608/fp64_hadamard/v0": 7.25e+08,
    "tet_p2_tgv_196608/fp64_split/v0": 7.29e+08,
    "tet_p2_tgv_196608/fp64_split/v1": 7.296e+08,
    "tet_p2_tgv_196608/fp64_vjp/v0": 3.121e+09,
    "tet_p2_tgv_196608/fp64_vjp/v1": 1.34e+09,
    "tet_p2_tgv_196608_curved/fp32_split/v0": 7.267e+08,
    "tet_p2_tgv_196608_curved/fp64_hadamard/v0": 7.22e+08,
    "tet_p2_tgv_196608_curved/fp64_split/v0": 7.618e+08,
    "tet_p2_tgv_196608_curved/fp64_vjp/v0": 1.373e+09,
    "tet_p2_tgv_196608_curved/fp64_vjp/v1": 5.8e+09,
    "tet_p3_tgv_196608/fp32_split/v0": 1.147e+09,
    "tet_p3_tgv_196608/fp32_split/v1": 1.192e+09,
    "tet_p3_tgv_196608/fp64_hadamard/v0": 1.242e+09,
    "tet_p3_tgv_196608/fp64_split/v0": 1.393e+09,
    "tet_p3_tgv_196608/fp64_split/v1": 1.386e+09,
    "tet_p3_tgv_196608/fp64_vjp/v0": 6.811e+09,
    "tet_p3_tgv_196608/fp64_vjp/v1": 2.419e+09,
    "tet_p3_tgv_196608_curved/fp32_split/v0": 1.181e+09,
    "tet_p3_tgv_196608_curved/fp64_hadamard/v0": 1.276e+09,
    "tet_p3_tgv_196608_curved/fp64_split/v0": 1.426e+09,
    "tet_p3_tgv_196608_curved/fp64_vjp/v0": 2.453e+09,
    "tet_p3_tgv_196608_curved/fp64_vjp/v1": 1.413e+10,
    "tri_batch4/fwd/v0": 1.437e+08,
    "tri_p1/fp32_split/v0": 2.244e+07,
    "tri_p1/fp32_split/v1": 2.246e+07,
    "tri_p1/fp32_split/v2": 2.23e+07,
    "tri_p1/fp64_hadamard/v0": 2.603e+07,
    "tri_p1/fp64_hadamard_vjp/v0": 4.681e+07,
    "tri_p1/fp64_split/v0": 2.556e+07,
    "tri_p1/fp64_split/v1": 1.73e+07,
    "tri_p1/fp64_split/v2": 2.601e+07,
    "tri_p1/fp64_vjp/v0": 1.238e+08,
    "tri_p1/fp64_vjp/v1": 4.688e+07,
    "tri_p2/fp32_split/v0": 3.562e+07,
    "tri_p2/fp32_split/v1": 2.106e+07,
    "tri_p2/fp32_split/v2": 3.355e+07,
    "tri_p2/fp64_hadamard/v0": 4.084e+07,
    "tri_p2/fp64_hadamard_vjp/v0": 7.22e+07,
    "tri_p2/fp64_split/v0": 2.65e+07,
    "tri_p2/fp64_split/v1": 2.636e+07,
    "tri_p2/fp64_split/v2": 2.672e+07,
    "tri_p2/fp64_vjp/v0": 7.502e+07,
    "tri_p2/fp64_vjp/v1": 7.224e+07,
    "tri_p3/fp32_split/v0": 3.536e+07,
    "tri_p3/fp32_split/v1": 3.445e+07,
    "tri_p3/fp32_split/v2": 3.455e+07,
    "tri_p3/fp64_hadamard/v0": 6.654e+07,
    "tri_p3/fp64_hadamard_vjp/v0": 1.182e+08,
    "tri_p3/fp64_split/v0": 4.413e+07,
    "tri_p3/fp64_split/v1": 4.397e+07,
    "tri_p3/fp64_split/v2": 4.437e+07,
    "tri_p3/fp64_vjp/v0": 1.214e+08,
    "tri_p3/fp64_vjp/v1": 1.183e+08,
    "tri_p4/fp32_split/v0": 4.282e+07,
    "tri_p4/fp32_split/v1": 4.141e+07,
    "tri_p4/fp32_split/v2": 4.15e+07,
    "tri_p4/fp64_hadamard/v0": 7.07e+07,
    "tri_p4/fp64_hadamard_vjp/v0": 1.215e+08,
    "tri_p4/fp64_split/v0": 5.319e+07,
    "tri_p4/fp64_split/v1": 5.304e+07,
    "tri_p4/fp64_split/v2": 5.413e+07,
    "tri_p4/fp64_vjp/v0": 1.248e+08,
    "tri_p4/fp64_vjp/v1": 1.216e+08,
}
KERNEL_SOURCES = ["residual_kernels.hip", "vjp_kernels.hip", "rrk_kernels.hip", "device_physics.hpp",
                  "mfma.hpp", "kernels.hpp"]

POINTWISE_FLOPS_PER_NODE = 500.0      # primitives, W, fluxes, A~ g, facet SAT share
VISCOUS_POINTWISE_PER_NODE = 150.0    # F^V from the gradients, BO facet terms
TWO_POINT_FLUX_FLOPS = 175.0          # one Sjoegren-Yee two-point flux (all directions)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-ms", type=float, default=200.0,
                    help="untimed setup: back-to-back headline calls for this long before tuning and warmup")
    ap.add_argument("--no-extras", action="store_true",
                    help="report only the headline step (used under a profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in launch shapes (skip sbp_autotune during setup)")
    ap.add_argument("--only", default=None,
                    help="run one breakdown family only and print it (tri, jitter, tet, tet_curved, ns, "
                         "hybrid, batch)")
    ap.add_argument("--probe-kernels", default=None, metavar="FILE",
                    help="run every timed call once per kernel variant between marker kernels and "
                         "write the call list to FILE (for counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy three times (calibrates HBM byte counters)")
    return ap.parse_args()


def kernel_source_hash():
    """sha256 (16 hex digits) of the kernel sources without their // comments
    and blank lines: a change of the code, not of its comments, voids the
    counter figures."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_07181_amd", "csrc", f)) as fh:
            code = re.sub(r"//[^\n]*", "", fh.read())
        h.update("\n".join(l.rstrip() for l in code.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(key, variant):
    """Counter-measured HBM bytes per call for the row key and kernel
    variant, or None if not measured on these kernel sources."""
    if not TRAFFIC or kernel_source_hash() != TRAFFIC_SHA:
        return None
    return TRAFFIC.get(f"{key}/v{variant}")


# ----------------------------------------------------------------------------
# algorithmic work per element (flops, HBM bytes)
# ----------------------------------------------------------------------------

def _geo_bytes(dim, curved):
    if dim == 2:
        return 12 * 8              # six quadratic map nodes
    return (30 if curved else 10) * 8   # ten map nodes, or Lambda (9) and J


def work_split(dim, n_p, n_f, out_bytes=8, curved=False):
    """Entropy split (Euler terms): 4 d n_c n_p^2 operator flops (one [c_b Q +
    Q^T] and one D application per direction and component) plus 500 flops
    per node of pointwise work; bytes: read u, write r, the map or metric
    data, the face-node map (4 B per facet node) and the element offset."""
    n_c = dim + 2
    flops = 4.0 * dim * n_c * n_p * n_p + POINTWISE_FLOPS_PER_NODE * n_p
    byts = n_c * n_p * (8 + out_bytes) + _geo_bytes(dim, curved) + (dim + 1) * n_f * 4 + 4
    return flops, byts


def work_hadamard(dim, n_p, n_f, curved=False):
    """Hadamard form: one two-point flux (175 flops, all directions) per node
    pair, 2 d n_c n_p^2 flops of S contraction, the pointwise and facet work of
    the split form; the same bytes."""
    n_c = dim + 2
    flops = (TWO_POINT_FLUX_FLOPS * n_p * (n_p - 1) / 2 + 2.0 * dim * n_c * n_p * n_p
             + POINTWISE_FLOPS_PER_NODE * n_p)
    return flops, work_split(dim, n_p, n_f, 8, curved)[1]


def work_vjp(fwd_flops, dim, n_p, n_f, curved=False):
    """VJP: twice the forward flops (the forward pass recomputed plus one
    transposed application of every operator); bytes: read u and lambda,
    write u-bar, the map or metric data and the face-node map."""
    n_c = dim + 2
    byts = 3 * n_c * n_p * 8 + _geo_bytes(dim, curved) + (dim + 1) * n_f * 4 + 4
    return 2.0 * fwd_flops, byts


def work_ns(n_p, n_f, out_bytes=8):
    """Navier-Stokes residual on affine tetrahedra: the Euler split terms plus
    2 d n_c n_p^2 for the gradient D_x w, 2 d n_c n_p^2 for D_x^T F^V, 2 n_p
    n_fac n_f d n_c for the facet-supported transposed derivatives, and 150
    flops per node for F^V and the BO facet terms; bytes as the split form
    (the facet exchange of n.F^V between the two kernels is implementation
    traffic, counted by the counters only)."""
    dim, n_c, n_fac = 3, 5, 4
    fl, by = work_split(dim, n_p, n_f, out_bytes)
    fl += 4.0 * dim * n_c * n_p * n_p + 2.0 * n_p * n_fac * n_f * dim * n_c + VISCOUS_POINTWISE_PER_NODE * n_p
    return fl, by


def roofline(fl, by, n_elem, sec, peak_flops, compute_bound, key, variant, kernel):
    """The roofline object of one timed call: bound = whichever of flops/peak
    and bytes/HBM peak is longer; achieved in that bound's unit."""
    t_c = fl * n_elem / peak_flops
    t_m = by * n_elem / PEAK_HBM
    if t_c >= t_m:
        r = dict(bound=compute_bound, achieved=fl * n_elem / sec / 1e12, peak=peak_flops / 1e12, unit="TFLOP/s")
    else:
        r = dict(bound="hbm", achieved=by * n_elem / sec / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s")
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = measured_traffic(key, variant)
    r["algorithmic_bytes"] = by * n_elem
    r["kernel"] = kernel
    r["avg_launch_ms"] = sec * 1e3
    r["work_per_element"] = dict(flops=fl, bytes=by)
    return r


# ----------------------------------------------------------------------------
# states and timing
# ----------------------------------------------------------------------------

def _state_from_mesh(mesh, kind, seed=0, jitter=0.0, L=20.0):
    import torch
    from paper_2305_07181_amd import workloads as wl
    x = mesh.node_coords().cpu().numpy()
    n_p = int(mesh.elem_np[0])
    X = np.moveaxis(x.reshape(mesh.n_elem, mesh.dim, n_p), 1, 0)
    if kind == "vortex":
        rho, V, p = wl.isentropic_vortex(X)
    elif kind == "tgv":
        rho, V, p = wl.taylor_green(X)
    elif kind == "random":
        rho, V, p = wl.random_smooth_state(X, seed=seed, L=L)
    else:
        raise ValueError(kind)
    u = np.moveaxis(wl.conservative(rho, V, p), 0, 1)
    if jitter:
        # independent node values on the two sides of every facet
        u = u * (1.0 + jitter * np.random.default_rng(seed + 7).standard_normal(u.shape))
    return torch.from_numpy(np.ascontiguousarray(u)).cuda()


def headline_mesh(desc, ps):
    """One mesh of len(ps) independent copies of the grid `desc`, copy b of
    degree ps[b] (a mesh of several degree classes: one batched launch per
    residual), and the vortex state on it."""
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    d4, deg, off = wl.copies_mesh(desc, ps)
    mesh = sbp.Mesh(d4, deg, problem_off=off)
    x = mesh.node_coords().cpu().numpy()
    u = np.zeros(int(mesh.n_nodes * mesh.n_c))
    for b in range(len(ps)):
        n_p = int(mesh.elem_np[off[b]])
        e0, e1 = int(off[b]), int(off[b + 1])
        lo, hi = int(mesh.node_off[e0]), int(mesh.node_off[e1])
        X = np.moveaxis(x[lo * 2:hi * 2].reshape(e1 - e0, 2, n_p), 1, 0)
        rho, V, pr = wl.isentropic_vortex(X)
        u[lo * 4:hi * 4] = np.moveaxis(wl.conservative(rho, V, pr), 0, 1).ravel()
    return mesh, torch.from_numpy(u).cuda()


def _tune(args, mesh, u, lam=None):
    """sbp_autotune during setup (untimed): the launch shapes it keeps."""
    if args.no_tune:
        return []
    return [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in t.items()}
            for t in mesh.autotune(u, lam)]


def _settle(fn, ms):
    """Back-to-back calls of `fn` for about `ms` milliseconds (untimed setup;
    returns the number of calls).  The device's clocks and caches reach their
    steady state only under sustained load: without it a run of 20 steps of
    0.12 ms read its kernel 4% slower than runs of 200 or 1000 steps."""
    import time
    import torch
    n = 0
    if ms <= 0:
        return n
    end = time.perf_counter() + ms * 1e-3
    while time.perf_counter() < end:
        for _ in range(50):
            fn()
        torch.cuda.synchronize()
        n += 50
    return n


def _time_calls(fn, reps, warm):
    """Mean duration of one call over `reps` back-to-back calls between two
    HIP events on torch's current stream (the stream the library launches
    on); events around every single call would add an event packet and its
    dispatch gap (about 6 us on MI355X) to each."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3 / reps
    return float(t), float(t)


def _variant(mesh, kind, p):
    try:
        return mesh.launch_shape(kind, p)[0]
    except Exception:
        return 0


def _fp32_error(r32, r64):
    """Per conserved component: max |r32 - r64| / max |r64| over the mesh
    (r64: the FP64 GPU residual, parity-tested against the FP64 oracle),
    computed on the host from copies of both (no device-side conversion)."""
    a = r32.cpu().numpy().astype(np.float64)
    b = r64.cpu().numpy()
    return [float(v) for v in np.abs(a - b).max(axis=(0, 2)) / np.abs(b).max(axis=(0, 2))]


class Runner:
    """Times calls (or, in probe mode, runs each once per kernel variant
    between marker kernels for counter runs)."""

    def __init__(self, args):
        self.args = args
        self.probe = args.probe_kernels is not None
        self.calls = []

    def reps(self, big=False):
        return 5 if big else max(10, self.args.steps)

    def measure(self, key, fn, mesh=None, slot=None, big=False):
        """Median call time (timing mode) or marker-bracketed probe runs; slot
        = (kind, p) of the launch shape to sweep in probe mode."""
        import torch
        if not self.probe:
            med, _ = _time_calls(fn, self.reps(big), 2)
            return med
        nvar = 1
        v0 = g0 = None
        if mesh is not None and slot is not None:
            v0, g0 = mesh.launch_shape(*slot)
            nvar = 1
            while True:
                try:
                    mesh.set_launch_shape(slot[0], slot[1], nvar, g0)
                    nvar += 1
                except Exception:
                    break
        print(f"[probe] {key} ({nvar} variant{'s' if nvar > 1 else ''})", file=sys.stderr, flush=True)
        for v in range(nvar):
            if nvar > 1:
                mesh.set_launch_shape(slot[0], slot[1], v, g0)
            fn()                                    # warm (first-call setup outside the markers)
            torch.cuda.synchronize()
            torch.cuda._sleep(1000)                 # marker
            fn()
            torch.cuda._sleep(1000)                 # marker
            torch.cuda.synchronize()
            self.calls.append(f"{key}/v{v}")
        if nvar > 1:
            mesh.set_launch_shape(slot[0], slot[1], v0, g0)
        return float("nan")

    def write(self):
        with open(self.args.probe_kernels, "w") as f:
            json.dump(dict(source_hash=kernel_source_hash(), calls=self.calls), f, indent=1)


def _variant_times(R, mesh, slot, fn, big):
    """Launch time of every kernel variant of a slot at its kept grid (the
    tuner keeps the fastest; this shows the alternatives, e.g. the register
    budget of one wave per SIMD without spills against two waves with)."""
    v0, g0 = mesh.launch_shape(*slot)
    out = {}
    v = 0
    while True:
        try:
            mesh.set_launch_shape(slot[0], slot[1], v, g0)
        except Exception:
            break
        out[f"v{v}"], _ = _time_calls(fn, R.reps(big), 2)
        out[f"v{v}"] *= 1e3
        v += 1
    mesh.set_launch_shape(slot[0], slot[1], v0, g0)
    return out


def _row(R, key, name, fn, mesh, slot, work, n_elem, n_p, peak, bound, kernel, big=False, variants=False):
    sec = R.measure(f"{key}/{name}", fn, mesh, slot, big)
    var = _variant(mesh, *slot) if slot else 0
    row = dict(ms=sec * 1e3, elem_dof_per_s=n_elem * n_p / sec,
               roofline=roofline(work[0], work[1], n_elem, sec, peak, bound, f"{key}/{name}", var, kernel))
    if variants and slot and not R.probe:
        row["variant_ms"] = _variant_times(R, mesh, slot, fn, big)
        row["variant_kept"] = var
    return row


# ----------------------------------------------------------------------------
# breakdown families
# ----------------------------------------------------------------------------

def tri_rows(R, desc, meshes, states, lams):
    """32768 curved triangles, vortex state, p = 1..4: FP64 and FP32 entropy
    split, the Hadamard form and its VJP, the VJP; FP32 error."""
    import torch
    from paper_2305_07181_amd import sbp
    ne = len(desc["elem_vert"])
    out = {}
    for p in sorted(meshes):
        m64, u, lam = meshes[p], states[p], lams[p]
        n_p = int(m64.elem_np[0])
        n_f = sbp.reference_operator(2, p)["n_f"]
        row = {}
        r64 = torch.empty_like(u)
        ws = work_split(2, n_p, n_f)
        row["fp64_split"] = _row(R, f"tri_p{p}", "fp64_split", lambda: m64.residual(u, r64), m64, ("residual", p),
                                 ws, ne, n_p, PEAK_F64, "alu", f"k_split2<{p},double,*> (vector ALU)")
        m64.residual(u, r64)
        m32 = sbp.Mesh(desc, p, precision=sbp.FP32)
        row["tuned_fp32"] = _tune(R.args, m32, u)
        r32 = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        row["fp32_split"] = _row(R, f"tri_p{p}", "fp32_split", lambda: m32.residual(u, r32), m32, ("residual", p),
                                 work_split(2, n_p, n_f, 4), ne, n_p, PEAK_F32, "alu",
                                 f"k_split2<{p},float,*> (vector ALU)")
        m32.residual(u, r32)
        row["fp32_rel_err_per_component"] = _fp32_error(r32, r64)
        m32.close()
        mh = sbp.Mesh(desc, p, form=sbp.FORM_HADAMARD)
        row["tuned_hadamard"] = _tune(R.args, mh, u)
        rh = torch.empty_like(u)
        wh = work_hadamard(2, n_p, n_f)
        row["fp64_hadamard"] = _row(R, f"tri_p{p}", "fp64_hadamard", lambda: mh.residual(u, rh), mh, None,
                                    wh, ne, n_p, PEAK_F64, "alu", f"k_hadamard<2,{p},double> (vector ALU)")
        ubh = torch.empty_like(u)
        row["fp64_hadamard_vjp"] = _row(R, f"tri_p{p}", "fp64_hadamard_vjp", lambda: mh.vjp(u, lam, ubh), mh, None,
                                        work_vjp(wh[0], 2, n_p, n_f), ne, n_p, PEAK_F64, "alu",
                                        f"k_vjp_had<2,{p}> (vector ALU)")
        mh.close()
        ub = torch.empty_like(u)
        row["fp64_vjp"] = _row(R, f"tri_p{p}", "fp64_vjp", lambda: m64.vjp(u, lam, ub), m64, ("vjp", p),
                               work_vjp(ws[0], 2, n_p, n_f), ne, n_p, PEAK_F64, "alu",
                               f"k_vjp2<{p},*> (vector ALU)", variants=True)
        row["hadamard_over_split"] = row["fp64_hadamard"]["ms"] / row["fp64_split"]["ms"]
        row["fp32_speedup"] = row["fp64_split"]["ms"] / row["fp32_split"]["ms"]
        row["vjp_over_forward"] = row["fp64_vjp"]["ms"] / row["fp64_split"]["ms"]
        out[f"tri_p{p}"] = row
        del r64, r32, rh, ubh, ub
    return out


def jitter_rows(R, desc):
    """The same 32768 triangles with a random smooth state (seed 0) whose node
    values carry 1% independent noise (seed 7): the two sides of every facet
    differ, so the exponential averages take their direct (logarithm) branch
    wherever the jump is large; FP64 split, p = 1..4, and the FP32 error on
    this state (whose residual is of the size of its terms)."""
    import torch
    from paper_2305_07181_amd import sbp
    ne = len(desc["elem_vert"])
    out = dict(state="random smooth (seed 0) x (1 + 0.01 N(0,1)) per node value (seed 7)")
    for p in (1, 2, 3, 4):
        m = sbp.Mesh(desc, p)
        u = _state_from_mesh(m, "random", seed=0, jitter=0.01)
        tuned = _tune(R.args, m, u)
        n_p = int(m.elem_np[0])
        n_f = sbp.reference_operator(2, p)["n_f"]
        r = torch.empty_like(u)
        row = _row(R, f"jitter_p{p}", "fp64_split", lambda: m.residual(u, r), m, ("residual", p),
                   work_split(2, n_p, n_f), ne, n_p, PEAK_F64, "alu", f"k_split2<{p},double,*> (vector ALU)")
        row["tuned"] = tuned
        m.residual(u, r)
        m32 = sbp.Mesh(desc, p, precision=sbp.FP32)
        row["fp32_rel_err_per_component"] = _fp32_error(m32.residual(u), r)
        m32.close()
        m.check_device()
        m.close()
        out[f"p{p}"] = row
    return out


def tet_rows(R, curved):
    """Taylor-Green (M = 0.1) on 32^3 x 6 = 196608 tetrahedra, p = 2, 3,
    matrix dissipation; affine or with quadratic maps (warp 0.02): FP64 and
    FP32 split, Hadamard form, VJP; FP32 error."""
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    desc = wl.curved_tet_mesh(32, 2.0 * np.pi, 0.02) if curved else wl.tgv_mesh(32)
    ne = len(desc["elem_vert"])
    kname = "k_split3c" if curved else "k_split3v"
    out = {}
    for p in (2, 3):
        key = f"tet_p{p}_tgv_196608" + ("_curved" if curved else "")
        row = {}
        m64 = sbp.Mesh(desc, p, dissipation=True)
        u = _state_from_mesh(m64, "tgv")
        n_p = int(m64.elem_np[0])
        n_f = sbp.reference_operator(3, p)["n_f"]
        lam = torch.randn(u.shape, dtype=torch.float64, device="cuda",
                          generator=torch.Generator(device="cuda").manual_seed(2100 + p))
        row["tuned_fp64"] = _tune(R.args, m64, u, lam)
        r64 = torch.empty_like(u)
        ws = work_split(3, n_p, n_f, 8, curved)
        row["fp64_split"] = _row(R, key, "fp64_split", lambda: m64.residual(u, r64), m64, ("residual", p), ws,
                                 ne, n_p, PEAK_F64, "alu", f"{kname}<{p},double> (vector ALU)", big=True)
        m64.residual(u, r64)
        ub = torch.empty_like(u)
        row["fp64_vjp"] = _row(R, key, "fp64_vjp", lambda: m64.vjp(u, lam, ub), m64, ("vjp", p),
                               work_vjp(ws[0], 3, n_p, n_f, curved), ne, n_p, PEAK_F64, "alu",
                               f"{'k_vjp3c' if curved else 'k_vjp3v'}<{p},*> (vector ALU)", big=True,
                               variants=True)
        del ub, lam
        m32 = sbp.Mesh(desc, p, dissipation=True, precision=sbp.FP32)
        row["tuned_fp32"] = _tune(R.args, m32, u)
        r32 = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        row["fp32_split"] = _row(R, key, "fp32_split", lambda: m32.residual(u, r32), m32, ("residual", p),
                                 work_split(3, n_p, n_f, 4, curved), ne, n_p, PEAK_F32, "alu",
                                 f"{kname}<{p},float> (vector ALU)", big=True)
        m32.residual(u, r32)
        row["fp32_rel_err_per_component"] = _fp32_error(r32, r64)
        uj = _state_from_mesh(m64, "random", seed=0, jitter=0.01, L=2.0 * np.pi)
        row["fp32_rel_err_per_component_jittered"] = _fp32_error(m32.residual(uj), m64.residual(uj))
        m32.close()
        del r32, uj
        mh = sbp.Mesh(desc, p, dissipation=True, form=sbp.FORM_HADAMARD)
        row["tuned_hadamard"] = _tune(R.args, mh, u)
        rh = torch.empty_like(u)
        row["fp64_hadamard"] = _row(R, key, "fp64_hadamard", lambda: mh.residual(u, rh), mh, None,
                                    work_hadamard(3, n_p, n_f, curved), ne, n_p, PEAK_F64, "alu",
                                    f"k_hadamard<3,{p},double,{'true' if curved else 'false'}> (vector ALU)",
                                    big=True)
        mh.check_device()
        mh.close()
        m64.check_device()
        m64.close()
        del rh, r64, u
        row["hadamard_over_split"] = row["fp64_hadamard"]["ms"] / row["fp64_split"]["ms"]
        row["fp32_speedup"] = row["fp64_split"]["ms"] / row["fp32_split"]["ms"]
        row["vjp_over_forward"] = row["fp64_vjp"]["ms"] / row["fp64_split"]["ms"]
        out[key] = row
    return out


def ns_rows(R):
    """Navier-Stokes Taylor-Green vortex on 24^3 x 6 = 82944 tetrahedra, p = 3,
    M = 0.1, Re = 1600, Pr = 0.71, heat flux and matrix dissipation on: the
    residual in FP64 and FP32 (FP32 error), the FP64 VJP, and RRK4 steps
    (FP32 and FP64 residuals, FP64 state and relaxation) replayed as one
    captured graph and launched eagerly."""
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    desc = wl.tgv_mesh(24)
    ne = len(desc["elem_vert"])
    kw = dict(dissipation=True, viscous=True, heat_flux=True, mu=1.0 / 1600, Pr=0.71, R=1.0)
    row = dict(n_elem=ne)
    m64 = sbp.Mesh(desc, 3, **kw)
    u = _state_from_mesh(m64, "tgv")
    n_p = int(m64.elem_np[0])
    n_f = sbp.reference_operator(3, 3)["n_f"]
    row["tuned_fp64"] = _tune(R.args, m64, u)
    r64 = torch.empty_like(u)
    wn = work_ns(n_p, n_f)
    row["fp64_residual"] = _row(R, "ns_tgv_82944_p3", "fp64_residual", lambda: m64.residual(u, r64), m64,
                                ("residual", 3), wn, ne, n_p, PEAK_F64, "mfma",
                                "k_visc_q3<3,double> + k_split3<3,double,true> (FP64 MFMA)", big=True)
    m64.residual(u, r64)
    lam = torch.randn(u.shape, dtype=torch.float64, device="cuda",
                      generator=torch.Generator(device="cuda").manual_seed(2300))
    ub = torch.empty_like(u)
    row["fp64_vjp"] = _row(R, "ns_tgv_82944_p3", "fp64_vjp", lambda: m64.vjp(u, lam, ub), m64, None,
                           work_vjp(wn[0], 3, n_p, n_f), ne, n_p, PEAK_F64, "alu",
                           "k_vjp3v<3,*> + k_vjpv_pre + k_vjpv (vector ALU)", big=True)
    row["vjp_over_forward"] = row["fp64_vjp"]["ms"] / row["fp64_residual"]["ms"]
    del ub, lam
    m32 = sbp.Mesh(desc, 3, precision=sbp.FP32, **kw)
    row["tuned_fp32"] = _tune(R.args, m32, u)
    r32 = torch.empty(u.shape, dtype=torch.float32, device="cuda")
    row["fp32_residual"] = _row(R, "ns_tgv_82944_p3", "fp32_residual", lambda: m32.residual(u, r32), m32,
                                ("residual", 3), work_ns(n_p, n_f, 4), ne, n_p, PEAK_F32, "mfma",
                                "k_visc_q3<3,float> + k_split3<3,float,true> (FP32 MFMA)", big=True)
    m32.residual(u, r32)
    row["fp32_rel_err_per_component"] = _fp32_error(r32, r64)
    uj = _state_from_mesh(m64, "random", seed=0, jitter=0.01, L=2.0 * np.pi)
    row["fp32_rel_err_per_component_jittered"] = _fp32_error(m32.residual(uj), m64.residual(uj))
    del uj
    row["fp32_speedup"] = row["fp64_residual"]["ms"] / row["fp32_residual"]["ms"]
    m64.close()
    del r32, r64
    if R.probe:
        m32.close()
        return row
    for name, m in (("fp32", m32), ("fp64", sbp.Mesh(desc, 3, **kw))):
        if name == "fp64":
            _tune(R.args, m, u)
        for mode in ("graph", "eager"):
            m.use_graphs(mode == "graph")
            uu = u.clone()
            m.rrk_step(uu, cfl=0.5)                    # warm-up (and capture)
            torch.cuda.synchronize()
            reps = []
            t0 = time.perf_counter()
            for _ in range(10):
                reps.append(m.rrk_step(uu, cfl=0.5))
            torch.cuda.synchronize()
            row[f"rrk_step_{name}_{mode}_ms"] = (time.perf_counter() - t0) / 10 * 1e3
            m.rrk_step(uu, cfl=0.5, report=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                m.rrk_step(uu, cfl=0.5, report=False)
            torch.cuda.synchronize()
            row[f"rrk_step_{name}_{mode}_noreport_ms"] = (time.perf_counter() - t0) / 10 * 1e3
            if mode == "graph":
                row[f"rrk_{name}"] = dict(
                    newton_iters_mean=float(np.mean([q["iters"] for q in reps])),
                    gamma_min=float(min(q["gamma"] for q in reps)), gamma_max=float(max(q["gamma"] for q in reps)),
                    entropy_nonincreasing=bool(all(q["entropy_after"] <= q["entropy_before"] for q in reps)),
                    dt=float(reps[-1]["dt"]))
        m.close()
    # the history of the Taylor-Green study over 100 steps at CFL 0.1
    # (Sec. 7.5): scaled kinetic energy, dissipation rate, total entropy
    from paper_2305_07181_amd import studies
    h = studies.tgv_run(24, 3, steps=100, re=1600.0, cfl=0.1)
    row["history_100_steps"] = dict(cfl=0.1, seconds=h["seconds"], t_end=h["t"][-1], E_k_start=h["E_k"][0],
                                    E_k_end=h["E_k"][-1], epsilon_min=min(h["epsilon"]),
                                    epsilon_max=max(h["epsilon"]), epsilon_incompressible_t0=3.0 / (4.0 * 1600.0),
                                    entropy_change_rel=(h["entropy"][-1] - h["entropy"][0]) / abs(h["entropy"][0]))
    return row


def rrk2d_rows(R, mesh, u):
    """RRK4 steps on the 32768-triangle mesh at p = 4 (FP64, EC SATs): short
    residuals, so launch overhead is visible; captured graph against eager
    launches, with and without the report's entropy sums."""
    import torch
    row = {}
    if R.probe:
        return row
    for mode in ("graph", "eager"):
        mesh.use_graphs(mode == "graph")
        for rep in (True, False):
            uu = u.clone()
            mesh.rrk_step(uu, cfl=0.1, report=rep)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                mesh.rrk_step(uu, cfl=0.1, report=rep)
            torch.cuda.synchronize()
            row[f"{mode}_{'report' if rep else 'noreport'}_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    mesh.use_graphs(True)
    row["eager_over_graph_noreport"] = row["eager_noreport_ms"] / row["graph_noreport_ms"]
    return row


def hybrid_rows(R, mesh, u, ne):
    """Hybrid scheme (Sec. 4.4) on the 32768-triangle mesh, p = 4: the
    residual with per-element flags -- a clustered region of the elements whose
    centroid lies in x < 2 (about 10%, where a shock detector would flag) and
    50% random flags (seed 7) -- against the pure split residual."""
    import torch
    if R.probe:
        return {}
    x = mesh.node_coords().cpu().numpy().reshape(ne, 2, -1).mean(axis=2)
    r = torch.empty_like(u)
    base, _ = _time_calls(lambda: mesh.residual(u, r), R.reps(), 2)
    row = dict(split_ms=base * 1e3)
    patterns = dict(clustered=(x[:, 0] < 2.0), random50=np.random.default_rng(7).random(ne) < 0.5)
    for name, sel in patterns.items():
        fd = torch.from_numpy(sel.astype(np.uint8)).cuda()
        mesh.set_volume_form(fd)
        med, _ = _time_calls(lambda: mesh.residual(u, r), R.reps(), 2)
        row[name] = dict(hadamard_elements=int(sel.sum()), ms=med * 1e3, over_split=med / base)
    mesh.set_volume_form(None)
    mesh.check_device()
    return row


def batch_rows(R):
    """48 independent periodic problems on [0,1]^2, p ~ U{1..4}, n_e ~ logU[256,
    16384] (seed 0), random smooth states (seed 1000+b): one batched forward
    launch and one batched VJP launch (lambda ~ N(0,1))."""
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    specs = wl.batch_problem_specs(48, 0)
    desc, deg, off = wl.batch_mesh(specs)
    mesh = sbp.Mesh(desc, deg, problem_off=off)
    x = mesh.node_coords().cpu().numpy()
    u = np.zeros(int(mesh.n_nodes * mesh.n_c))
    fl = by = flv = byv = 0.0
    for b, sp in enumerate(specs):
        n_p = int(mesh.elem_np[off[b]])
        e0, e1 = int(off[b]), int(off[b + 1])
        xs = x[int(mesh.node_off[e0]) * 2:int(mesh.node_off[e1]) * 2].reshape(e1 - e0, 2, n_p)
        rho, V, p = wl.random_smooth_state(np.moveaxis(xs, 1, 0), seed=1000 + b, L=1.0, K=4, amp=0.1, vamp=0.3)
        ub = np.moveaxis(wl.conservative(rho, V, p), 0, 1)
        u[int(mesh.node_off[e0]) * 4:int(mesh.node_off[e1]) * 4] = ub.ravel()
        f1, b1 = work_split(2, n_p, sbp.reference_operator(2, sp["p"])["n_f"])
        f2, b2 = work_vjp(f1, 2, n_p, sbp.reference_operator(2, sp["p"])["n_f"])
        fl += f1 * (e1 - e0)
        by += b1 * (e1 - e0)
        flv += f2 * (e1 - e0)
        byv += b2 * (e1 - e0)
    ud = torch.from_numpy(u).cuda()
    lam = torch.randn(ud.shape, dtype=torch.float64, device="cuda",
                      generator=torch.Generator(device="cuda").manual_seed(2000))
    r = torch.empty_like(ud)
    ubar = torch.empty_like(ud)
    tuned = _tune(R.args, mesh, ud, lam)
    ne = int(off[-1])
    ndof = int(mesh.n_nodes)
    fwd = _row(R, "batch48", "fwd", lambda: mesh.residual(ud, r), mesh, ("residual", 0), (fl / ne, by / ne), ne,
               ndof / ne, PEAK_F64, "alu", "k_split2_batch<double> (vector ALU, all degrees in one launch)")
    vjp = _row(R, "batch48", "vjp", lambda: mesh.vjp(ud, lam, ubar), mesh, ("vjp", 0), (flv / ne, byv / ne), ne,
               ndof / ne, PEAK_F64, "alu", "k_vjp2_batch (vector ALU, all degrees in one launch)")
    mesh.check_device()
    mesh.close()
    return dict(n_problems=48, n_elem=ne, n_dof_nodes=ndof,
                degrees={str(q): int(sum(1 for s in specs if s["p"] == q)) for q in (1, 2, 3, 4)},
                forward=fwd, vjp=vjp, vjp_over_forward=vjp["ms"] / fwd["ms"], tuned=tuned)


# ----------------------------------------------------------------------------
# CPU baseline: the oracle on the host's cores
# ----------------------------------------------------------------------------

def _cpu_setup(cfg, p, seed):
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import workloads as wl
    if cfg == "tri":
        desc = wl.vortex2d_mesh(128, warp=0.05)
        kind, diss = "vortex", False
    else:
        desc = wl.tgv_mesh(8)
        kind, diss = "tgv", True
    m = OracleMesh(desc, p)
    rng = np.random.default_rng(seed)
    els = rng.choice(m.ne, size=min(m.ne, 64), replace=False)
    need = set(int(e) for e in els)
    for e in list(need):
        for f in range(m.n_fac):
            need.add(m.neighbor(e, f)[0])
    need = sorted(need)
    X = np.moveaxis(m.node_coords(need), 1, 0)
    rho, V, pr = wl.isentropic_vortex(X) if kind == "vortex" else wl.taylor_green(X)
    u = np.zeros((m.ne, m.n_c, m.n_p))
    u[need] = np.moveaxis(wl.conservative(rho, V, pr), 0, 1)
    for e in need:
        m.geometry(e)                 # setup excluded from the timing (as in the paper)
    return OracleScheme(m, ph.Gas(), dissipation=diss), u, els


def _cpu_loop(sch, u, els, budget):
    n = 0
    t0 = time.perf_counter()
    while True:
        for e in els:
            sch.element(u, int(e))
            n += 1
        t1 = time.perf_counter()
        if t1 - t0 > budget:
            return n, t0, t1


def _cpu_worker(cfg, p, seed, budget, barrier, queue):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        sch, u, els = _cpu_setup(cfg, p, seed)
        barrier.wait(timeout=600)
        queue.put((cfg, p) + _cpu_loop(sch, u, els, budget))


def _cpu_all_cores(cfg, ps, cores, budget):
    """cores worker processes (one numpy thread each), cores / len(ps) per
    degree, each on its own sample of elements; set up, then timed together
    after a barrier.  Returns per p the core-seconds per element (busy time
    over elements, summed over its workers), the workers used and the
    window from the first start to the last end."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    per = max(1, cores // len(ps))
    barrier = ctx.Barrier(per * len(ps))
    queue = ctx.Queue()
    procs = [ctx.Process(target=_cpu_worker, args=(cfg, p, 100 * p + k, budget, barrier, queue))
             for p in ps for k in range(per)]
    for pr in procs:
        pr.start()
    import queue as _q
    res = []
    try:
        while len(res) < len(procs):
            try:
                res.append(queue.get(timeout=5))
            except _q.Empty:
                if any(pr.exitcode not in (None, 0) for pr in procs):
                    raise RuntimeError("a CPU baseline worker failed")
    finally:
        for pr in procs:
            if pr.is_alive() and len(res) < len(procs):
                pr.terminate()
            pr.join()
    t0 = min(r[3] for r in res)
    t1 = max(r[4] for r in res)
    out = {}
    for p in ps:
        n = sum(r[2] for r in res if r[1] == p)
        busy = sum(r[4] - r[3] for r in res if r[1] == p)
        out[p] = dict(core_sec_per_elem=busy / n, elems=n, workers=per)
    return out, per * len(ps), t1 - t0


def _cpu_one_core(cfg, ps, budget):
    from threadpoolctl import threadpool_limits
    out = {}
    with threadpool_limits(1):
        for p in ps:
            sch, u, els = _cpu_setup(cfg, p, 100 * p)
            n, t0, t1 = _cpu_loop(sch, u, els, budget)
            out[p] = dict(core_sec_per_elem=(t1 - t0) / n, elems=n, workers=1)
    return out


def cpu_baseline():
    """The oracle (plain numpy FP64, entropy split) timed on the host: all
    usable cores (at most 16: the host share of one GPU) as one process per
    core, and one core.  Per element times on samples of 64 elements per
    degree, scaled to elem-DOF/s of one residual of the whole mesh.  Config 2:
    32768 curved triangles, vortex, p = 1..4 (the headline workload); config
    3: tetrahedra with matrix dissipation, Taylor-Green, p = 2, 3 (elements of
    the 8^3 x 6 grid of the same family: the same per-element work as on the
    32^3 x 6 grid, without building the 196608-element oracle mesh)."""
    from oracle.operators import reference_operator
    cores = min(16, len(os.sched_getaffinity(0)))
    res = {}
    for cfg, ps, ne, dim, b_all, b_one in (("tri", (1, 2, 3, 4), 32768, 2, 8.0, 1.5),
                                           ("tet", (2, 3), 196608, 3, 5.0, 2.0)):
        allc, used, window = _cpu_all_cores(cfg, ps, cores, b_all)
        one = _cpu_one_core(cfg, ps, b_one)
        dofs = sum(ne * reference_operator(dim, p)["n_p"] for p in ps)
        core_sec = sum(allc[p]["core_sec_per_elem"] * ne for p in ps)
        res[cfg] = dict(value=dofs / (core_sec / used), cores=used, window_s=window,
                        one_core=dofs / sum(one[p]["core_sec_per_elem"] * ne for p in ps),
                        per_p={p: dict(all_cores=allc[p], one_core=one[p]) for p in ps})
    tri = res["tri"]
    return dict(value=tri["value"], unit="elem-DOF/s", cores=tri["cores"], kind="oracle",
                sample=f"oracle (numpy FP64, one thread per process) entropy-split residual of sampled "
                       f"elements (64 distinct per process and p, vortex state) of the 32768-triangle curved "
                       f"mesh, p = 1..4, {tri['cores']} processes timed together after a barrier for "
                       f"{tri['window_s']:.1f} s; core-seconds per element scaled to one residual per p of "
                       f"the whole mesh over the cores",
                one_core=dict(value=tri["one_core"], cores=1),
                config3_tet_tgv=dict(value=res["tet"]["value"], cores=res["tet"]["cores"],
                                     one_core=res["tet"]["one_core"], unit="elem-DOF/s",
                                     note="196608 tetrahedra, p = 2 and 3, dissipation on (per-element time "
                                          "on the 8^3 x 6 grid of the same family)"),
                per_p=dict(tri=res["tri"]["per_p"], tet=res["tet"]["per_p"]))


# ----------------------------------------------------------------------------

def main():
    args = _args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding "
              f"is a design only, not a measured path", file=sys.stderr)
        sys.exit(2)
    # the CPU oracle first, before the GPU is initialised (its worker
    # processes are started from a process that has not touched the GPU)
    cpu = None
    if not (args.no_cpu_baseline or args.probe_kernels or args.only):
        cpu = cpu_baseline()
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    assert torch.cuda.is_available()
    R = Runner(args)
    if args.only and args.only != "tri":
        fam = dict(jitter=lambda: jitter_rows(R, wl.vortex2d_mesh(128, warp=0.05)),
                   tet=lambda: tet_rows(R, False), tet_curved=lambda: tet_rows(R, True),
                   ns=lambda: ns_rows(R), batch=lambda: batch_rows(R))
        print(json.dumps({args.only: fam[args.only]()}))
        return
    ps = (1, 2, 3, 4)
    desc = wl.vortex2d_mesh(128, warp=0.05)
    ne = len(desc["elem_vert"])
    meshes, states, outs, lams, tuned = {}, {}, {}, {}, {}
    for p in ps:
        meshes[p] = sbp.Mesh(desc, p)
        states[p] = _state_from_mesh(meshes[p], "vortex")
        outs[p] = torch.empty_like(states[p])
        lams[p] = torch.randn(states[p].shape, dtype=torch.float64, device="cuda",
                              generator=torch.Generator(device="cuda").manual_seed(2000 + p))
    if not (args.no_tune or args.probe_kernels):
        _settle(lambda: meshes[4].residual(states[4], outs[4]), args.settle_ms)
    for p in ps:
        tuned[p] = _tune(args, meshes[p], states[p], lams[p])
    n_p = {p: int(meshes[p].elem_np[0]) for p in ps}
    dofs = sum(ne * n_p[p] for p in ps)
    if args.only == "tri":
        print(json.dumps({"tri": tri_rows(R, desc, meshes, states, lams)}))
        return

    # the headline step: the four degrees' residuals as one batched launch
    # (the four copies of the grid are independent problems of one mesh)
    mb, ub = headline_mesh(desc, ps)
    rb = torch.empty_like(ub)
    settle_calls = 0 if args.probe_kernels else _settle(lambda: mb.residual(ub, rb), args.settle_ms)
    tuned_b = _tune(args, mb, ub)
    ne_b = int(mb.n_elem)
    dofs = int(mb.n_nodes)
    assert dofs == sum(ne * n_p[p] for p in ps)

    if R.probe:
        R.measure("tri_batch4/fwd", lambda: mb.residual(ub, rb), mb, ("residual", 0))
        out = tri_rows(R, desc, meshes, states, lams)
        jitter_rows(R, desc)
        tet_rows(R, False)
        tet_rows(R, True)
        ns_rows(R)
        batch_rows(R)
        # calibration: a plain 256 MiB device copy between the markers
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        R.measure("copy_256MiB/read_write", lambda: dst.copy_(src))
        R.write()
        for p in ps:
            meshes[p].close()
        mb.close()
        print(json.dumps(dict(probe_calls=len(R.calls), source_hash=kernel_source_hash())))
        return

    for _ in range(args.warmup):
        mb.residual(ub, rb)
    torch.cuda.synchronize()
    # the step's one launch is timed inside the timed region by the kernel
    # itself (sbp_time_launches: its earliest workgroup start and latest
    # workgroup end on the device clock, no packets in the stream); two stream
    # events bracket the whole region
    mb.time_launches(args.steps)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        mb.residual(ub, rb)
    t1.record()
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1) * 1e-3
    ms_per_step = total / args.steps * 1e3
    value = dofs / (total / args.steps)
    ms = mb.launch_times(args.steps)
    mb.time_launches(0)
    assert len(ms) == args.steps
    kern_b = float(np.mean(ms)) * 1e-3
    mb.check_device()
    # each degree alone (its own mesh and launch), after the timed region
    kern = {}
    for p in ps:
        kern[p], _ = _time_calls(lambda: meshes[p].residual(states[p], outs[p]), max(10, args.steps), 2)
    fl = by = 0.0
    for p in ps:
        f1, b1 = work_split(2, n_p[p], sbp.reference_operator(2, p)["n_f"])
        fl += f1 * ne
        by += b1 * ne
    # the 2D kernel runs its pair sums and pointwise work on the FP64 vector
    # ALUs (256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s)
    roof = roofline(fl / ne_b, by / ne_b, ne_b, kern_b, PEAK_F64, "alu", "tri_batch4/fwd",
                    _variant(mb, "residual", 0),
                    f"k_split2_batch<double> (2D entropy split, the four degrees p = 1..4 of the 32768-triangle "
                    f"grid in one launch, {ne_b} elements)")
    roof["work_note"] = ("per element of each degree: 4 d n_c n_p^2 operator flops + 500 flops per node pointwise; "
                         "bytes: u, r, map nodes, face-node map, offset; work_per_element is the mean over the "
                         "four degrees")
    out = dict(metric=METRIC, value=value, unit="elem-DOF/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="2D Euler, curved periodic [0,20]^2 mesh 128x128x2 = 32768 triangles "
                                    "(P2 warp 0.05 L sin sin), isentropic vortex, entropy-split residual "
                                    "with EC SATs, FP64, one residual for each p = 1,2,3,4 per step, the four "
                                    "in one batched launch (one mesh of four independent copies of the grid)",
                           n_elem=ne, degrees=list(ps), n_p=n_p,
                           step_kernel_ms=kern_b * 1e3,
                           kernel_ms={p: kern[p] * 1e3 for p in ps},
                           kernel_ms_note="step_kernel_ms: mean duration of the step's one launch in the timed "
                                          "region (first workgroup start to last workgroup end, recorded by the "
                                          "kernel on the device clock); kernel_ms: each degree alone on its own "
                                          "mesh, mean of back-to-back launches after the timed region",
                           launch_shape=tuned_b,
                           launch_shapes={p: tuned[p] for p in ps},
                           settle=dict(ms=args.settle_ms, calls=settle_calls,
                                       note="untimed setup: back-to-back headline calls before tuning and "
                                            "warmup, for the device's steady state")),
               roofline=roof)
    if not args.no_extras:
        extras = tri_rows(R, desc, meshes, states, lams)
        extras["tri_jitter"] = jitter_rows(R, desc)
        extras.update(tet_rows(R, False))
        extras.update(tet_rows(R, True))
        for p in (2, 3):
            c, a = extras[f"tet_p{p}_tgv_196608_curved"], extras[f"tet_p{p}_tgv_196608"]
            c["curved_over_affine_fp64"] = c["fp64_split"]["ms"] / a["fp64_split"]["ms"]
            c["curved_over_affine_fp32"] = c["fp32_split"]["ms"] / a["fp32_split"]["ms"]
        extras["ns_tgv_82944_p3"] = ns_rows(R)
        extras["rrk_tri_p4_32768"] = rrk2d_rows(R, meshes[4], states[4])
        extras["hybrid_tri_p4"] = hybrid_rows(R, meshes[4], states[4], ne)
        extras["batch48"] = batch_rows(R)
        fw = sum(extras[f"tri_p{p}"]["fp64_split"]["ms"] for p in ps)
        bw = sum(extras[f"tri_p{p}"]["fp64_vjp"]["ms"] for p in ps)
        extras["vjp_over_forward"] = dict(
            headline=bw / fw, batch48=extras["batch48"]["vjp_over_forward"],
            ns_tgv_82944_p3=extras["ns_tgv_82944_p3"]["vjp_over_forward"],
            note="FP64 VJP time / FP64 residual time; headline = sum over p = 1..4 on the 32768-triangle mesh")
        k3 = ("tet_p2_tgv_196608", "tet_p3_tgv_196608", "tet_p2_tgv_196608_curved", "tet_p3_tgv_196608_curved",
              "ns_tgv_82944_p3")
        extras["fp32_rel_err_per_component"] = dict(
            jittered=dict({f"tri_p{p}": extras["tri_jitter"][f"p{p}"]["fp32_rel_err_per_component"] for p in ps},
                          **{k: extras[k]["fp32_rel_err_per_component_jittered"] for k in k3}),
            smooth=dict({f"tri_p{p}": extras[f"tri_p{p}"]["fp32_rel_err_per_component"] for p in ps},
                        **{k: extras[k]["fp32_rel_err_per_component"] for k in k3}),
            note="max |r_FP32 - r_FP64| / max |r_FP64| per conserved component over the whole mesh; r_FP64 is "
                 "the GPU FP64 residual (parity-tested against the FP64 oracle to 1e-12).  jittered: the random "
                 "smooth state with 1% node noise, whose residual is of the size of its terms; smooth: the "
                 "timed vortex / Taylor-Green states, whose residual is a small difference of large terms "
                 "(free stream, M = 0.1), so FP32 rounding of the terms dominates it")
        out["breakdown"] = extras
    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = dict(read=src.numel() * 8, write=dst.numel() * 8)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for p in ps:
        meshes[p].close()
    mb.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
