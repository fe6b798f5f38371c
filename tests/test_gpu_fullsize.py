"""Parity at the full sizes of the benchmark workloads, in the launch shapes
the benchmark times (the autotuner's choice on the same handle):

  * the curved periodic vortex grid, 128 x 128 x 2 = 32768 triangles, p = 1..4
    (split form in FP64 and FP32, Hadamard form, VJP);
  * the Taylor-Green grid, 32^3 x 6 = 196608 tetrahedra, p = 2, 3 with matrix
    dissipation (the same four);
  * the Navier-Stokes Taylor-Green grid, 24^3 x 6 = 82944 tetrahedra, p = 3,
    heat flux and matrix dissipation on (FP64 and FP32);
  * the 48-problem mixed-degree batch, 190202 triangles (residual, VJP and
    the finite-difference check of the whole batch).

The oracle evaluates sampled elements one by one (their facet neighbours'
states enter through the SATs); the inputs are the oracle's node coordinates
fed to the seeded workload generators, the same fields the benchmark uses.
The smooth states make the residual small against the terms summed into it
(free stream far from the vortex, low Mach number), so the error is taken
relative to the magnitude of those terms (term_scale), the scale of the
rounding of any evaluation order.  Properties of the whole grid: the entropy
rate vanishes without dissipation and is negative with it (Sec. 4).

On the same two grids a random smooth state with 1% independent noise on
every node value (the two sides of every facet differ, so the exponential
averages also take their logarithm branch) has no such cancellation, and
there the plain relative error per conserved component, max |r_gpu - r_orc|
/ max |r_orc| over the sampled nodes, is held to 1e-12."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state, term_scale

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-4
_cache = {}


def _workload(name, p, jitter=False):
    """(desc, OracleMesh, state) of one benchmark workload, kept for the
    tests of the same grid and degree; jitter: the random smooth state (seed
    0) with 1% independent noise on every node value (seed 7), so the two
    sides of every facet differ."""
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import workloads as wl
    key = (name, p)
    if key not in _cache:
        _cache.clear()
        desc = {"tri": lambda: wl.vortex2d_mesh(128, warp=0.05),
                "tet": lambda: wl.tgv_mesh(32),
                "ns": lambda: wl.tgv_mesh(24)}[name]()
        _cache[key] = (desc, OracleMesh(desc, p), {})
    desc, m, states = _cache[key]
    if jitter not in states:
        states[jitter] = (state(m, "random", seed=0, jitter=0.01) if jitter
                          else state(m, "vortex" if name == "tri" else "tgv"))
    return desc, m, states[jitter]


def _sample(ne, k, seed):
    rest = np.random.default_rng(seed).choice(np.arange(1, ne - 1), k - 2, replace=False)
    return [0, ne - 1] + sorted(int(e) for e in rest)


def _affine_H(m, ne):
    """H_k = h |det F_k| for affine elements, vectorised over the grid; pinned
    to the oracle's per-element geometry on a few elements."""
    v = m.verts[m.elem]                                          # [ne, d+1, d]
    F = np.stack([v[:, l + 1] - v[:, 0] for l in range(m.dim)], 2)
    H = np.abs(np.linalg.det(F))[:, None] * np.asarray(m.ops["h"])[None, :]
    for e in (0, ne // 3, ne - 1):
        assert np.allclose(H[e], m.geometry(e)["H"], rtol=1e-14, atol=0.0)
    return H


def _check_sampled(r, ro, sch, u, els, tol, what):
    sc = term_scale(sch, u, els)
    err = np.abs(np.asarray(r, dtype=np.float64)[els] - ro).max(axis=(0, 2)) / sc
    say(f"   {what}: max err / term scale {err.max():.2e} (per component {np.array2string(err, precision=1)})")
    assert (err <= tol).all(), (what, err)


def _tuned(mesh, ud, lamd=None):
    rep = mesh.autotune(ud, lamd)
    say("   tuned:", [(t["kind"], t["p"], t["variant"], t["grid"]) for t in rep])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tri32768_sampled(p):
    """The headline workload: each degree on the full curved triangle grid."""
    import torch
    from oracle import physics as ph
    from oracle.jacobian import vjp_elements
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[full tri32768] p={p}")
    desc, m, u = _workload("tri", p)
    ud = torch.from_numpy(u).cuda()
    lam = np.random.default_rng(2000 + p).standard_normal(u.shape)
    lamd = torch.from_numpy(lam).cuda()
    els = _sample(m.ne, 24, p)
    sch = OracleScheme(m, ph.Gas())
    ro = sch(u, elements=els)
    mesh = sbp.Mesh(desc, p)
    _tuned(mesh, ud, lamd)
    r, er = mesh.residual(ud, entropy_rate=True)
    mesh.check_device()
    r = r.cpu().numpy()
    _check_sampled(r, ro, sch, u, els, TOL64, "split FP64")
    # entropy conservation of the whole grid (no dissipation): w^T H r = 0
    # to the rounding of the sum of its terms
    w = ph.entropy_vars(np.moveaxis(u, 1, 0), sch.gas)          # [n_c, ne, n_p]
    H = m.H_all()                                                # curved maps: per element
    scale = float(np.sum(H[None] * np.abs(w) * np.abs(np.moveaxis(r, 1, 0))))
    say(f"   entropy rate {float(er.cpu()[0]):.3e}, scale {scale:.3e}")
    assert abs(float(er.cpu()[0])) <= 1e-12 * scale
    ub = mesh.vjp(ud, lamd).cpu().numpy()
    mesh.check_device()
    mesh.close()
    vel = els[:3]
    ref = vjp_elements(sch, u, lam, vel)
    sc = max(np.abs(ref[e]).max() for e in vel)
    err = max(np.abs(ub[e] - ref[e]).max() for e in vel) / sc
    say(f"   VJP rel err {err:.2e}")
    assert err <= TOL64, err
    for kw, tol, what, sch2 in ((dict(precision=sbp.FP32), TOL32, "split FP32", sch),
                                (dict(form=sbp.FORM_HADAMARD), TOL64, "Hadamard FP64",
                                 OracleScheme(m, ph.Gas(), form="hadamard"))):
        mesh = sbp.Mesh(desc, p, **kw)
        _tuned(mesh, ud)
        r = mesh.residual(ud)
        mesh.check_device()
        ro2 = ro if sch2 is sch else sch2(u, elements=els)
        _check_sampled(r.cpu().double().numpy(), ro2, sch2, u, els, tol, what)
        mesh.close()


@pytest.mark.parametrize("p,part", [(2, "residual"), (2, "vjp"), (3, "residual"), (3, "vjp")])
def test_tet196608_sampled(p, part):
    """The 3D Taylor-Green grid with matrix dissipation (the two parts of one
    degree run one after the other and share the oracle's grid)."""
    (_tet_residual if part == "residual" else _tet_vjp)(p)


def _tet_residual(p):
    """Split FP64 and FP32, Hadamard form, and the whole grid's entropy rate
    (negative)."""
    import torch
    from oracle import physics as ph
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[full tet196608] p={p}")
    desc, m, u = _workload("tet", p)
    ud = torch.from_numpy(u).cuda()
    els = _sample(m.ne, 12, 10 + p)
    sch = OracleScheme(m, ph.Gas(), dissipation=True)
    ro = sch(u, elements=els)
    mesh = sbp.Mesh(desc, p, dissipation=True)
    _tuned(mesh, ud)
    r, er = mesh.residual(ud, entropy_rate=True)
    mesh.check_device()
    _check_sampled(r.cpu().numpy(), ro, sch, u, els, TOL64, "split FP64")
    # the dissipation removes entropy; with H from the affine maps the grid's
    # rate recomputed from the GPU residual agrees with the fused one
    H = _affine_H(m, m.ne)
    w = ph.entropy_vars(np.moveaxis(u, 1, 0), sch.gas)
    rn = np.moveaxis(r.cpu().numpy(), 1, 0)
    rate = float(np.sum(H[None] * w * rn))
    scale = float(np.sum(H[None] * np.abs(w) * np.abs(rn)))
    rate_g = float(er.cpu()[0])
    say(f"   entropy rate {rate_g:.6e} (recomputed {rate:.6e}, scale {scale:.3e})")
    assert rate_g < 0 and abs(rate_g - rate) <= 1e-12 * scale
    mesh.close()
    for kw, tol, what, sch2 in ((dict(precision=sbp.FP32), TOL32, "split FP32", sch),
                                (dict(form=sbp.FORM_HADAMARD), TOL64, "Hadamard FP64",
                                 OracleScheme(m, ph.Gas(), form="hadamard", dissipation=True))):
        mesh = sbp.Mesh(desc, p, dissipation=True, **kw)
        _tuned(mesh, ud)
        r = mesh.residual(ud)
        mesh.check_device()
        ro2 = ro if sch2 is sch else sch2(u, elements=els)
        _check_sampled(r.cpu().double().numpy(), ro2, sch2, u, els, tol, what)
        mesh.close()


def _tet_vjp(p):
    """The VJP on the 3D Taylor-Green grid in its tuned launch shape against
    the oracle's complex-step Jacobian on sampled elements."""
    import torch
    from oracle import physics as ph
    from oracle.jacobian import vjp_elements
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[full tet196608 VJP] p={p}")
    desc, m, u = _workload("tet", p)
    ud = torch.from_numpy(u).cuda()
    lam = np.random.default_rng(2100 + p).standard_normal(u.shape)
    lamd = torch.from_numpy(lam).cuda()
    mesh = sbp.Mesh(desc, p, dissipation=True)
    _tuned(mesh, ud, lamd)
    ub = mesh.vjp(ud, lamd).cpu().numpy()
    mesh.check_device()
    mesh.close()
    vel = [0, m.ne - 1] if p == 2 else [m.ne // 2]
    ref = vjp_elements(OracleScheme(m, ph.Gas(), dissipation=True), u, lam, vel)
    sc = max(np.abs(ref[e]).max() for e in vel)
    err = max(np.abs(ub[e] - ref[e]).max() for e in vel) / sc
    say(f"   VJP rel err {err:.2e}")
    assert err <= TOL64, err


@pytest.mark.parametrize("kind,p", [("tri", 1), ("tri", 2), ("tri", 3), ("tri", 4), ("tet", 2), ("tet", 3)])
def test_jittered_state_plain_relative_error(kind, p):
    """Full grids (32768 curved triangles; 196608 tetrahedra with matrix
    dissipation), jittered random smooth state, tuned launch shapes: the
    entropy split and the Hadamard form in FP64 on sampled elements against
    the oracle, plain relative error per component <= 1e-12."""
    import torch
    from oracle import physics as ph
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[full jittered] {kind} p={p}")
    desc, m, u = _workload(kind, p, jitter=True)
    diss = kind == "tet"
    ud = torch.from_numpy(u).cuda()
    els = _sample(m.ne, 16 if kind == "tri" else 8, 40 + p)
    for form in ("split", "hadamard"):
        sch = OracleScheme(m, ph.Gas(), form=form, dissipation=diss)
        ro = sch(u, elements=els)
        mesh = sbp.Mesh(desc, p, dissipation=diss,
                        form=sbp.FORM_SPLIT if form == "split" else sbp.FORM_HADAMARD)
        _tuned(mesh, ud)
        r = mesh.residual(ud)
        mesh.check_device()
        mesh.close()
        err = rel_err_per_component(r.cpu().numpy()[els], ro)
        say(f"   {form}: plain rel err per component {np.array2string(err, precision=1)}")
        assert (err <= TOL64).all(), (form, err)


def test_headline_four_degrees_one_launch():
    """The benchmark's timed step: the 32768-triangle grid at p = 1..4 as four
    independent copies in one mesh (one batched launch), tuned as the
    benchmark does; sampled elements of every copy against the oracle (the
    summed-term scale of the smooth vortex state) and the entropy rate of the
    whole mesh (no dissipation: zero to rounding)."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[full headline, four degrees in one launch]")
    desc = wl.vortex2d_mesh(128, warp=0.05)
    ps = (1, 2, 3, 4)
    d4, deg, off = wl.copies_mesh(desc, ps)
    oms = {p: OracleMesh(desc, p) for p in ps}
    us = {p: state(oms[p], "vortex") for p in ps}
    mesh = sbp.Mesh(d4, deg, problem_off=off)
    nc = int(mesh.n_c)
    lo = [int(mesh.node_off[off[b]]) * nc for b in range(len(ps) + 1)]
    u = np.concatenate([us[p].ravel() for p in ps])
    assert all(lo[b + 1] - lo[b] == us[p].size for b, p in enumerate(ps))
    ud = torch.from_numpy(u).cuda()
    _tuned(mesh, ud)
    r, er = mesh.residual(ud, entropy_rate=True)
    mesh.check_device()
    r = r.cpu().numpy()
    scale = 0.0
    for b, p in enumerate(ps):
        m = oms[p]
        sch = OracleScheme(m, ph.Gas())
        els = _sample(m.ne, 12, 60 + p)
        ro = sch(us[p], elements=els)
        rp = r[lo[b]:lo[b + 1]].reshape(us[p].shape)
        _check_sampled(rp, ro, sch, us[p], els, TOL64, f"copy {b} p={p}")
        w = ph.entropy_vars(np.moveaxis(us[p], 1, 0), sch.gas)
        scale += float(np.sum(m.H_all()[None] * np.abs(w) * np.abs(np.moveaxis(rp, 1, 0))))
    say(f"   entropy rate {float(er.cpu()[0]):.3e}, scale {scale:.3e}")
    assert abs(float(er.cpu()[0])) <= 1e-12 * scale
    mesh.close()


def test_ns_tgv82944_sampled():
    """The Navier-Stokes Taylor-Green grid, p = 3, Re = 1600, Pr = 0.71, heat
    flux and matrix dissipation: FP64 and FP32 residuals on sampled elements."""
    import torch
    from oracle import physics as ph
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say("[full ns tgv82944] p=3")
    desc, m, u = _workload("ns", 3)
    ud = torch.from_numpy(u).cuda()
    els = _sample(m.ne, 8, 31)
    gas = ph.Gas(mu=1.0 / 1600, Pr=0.71, R=1.0)
    sch = OracleScheme(m, gas, dissipation=True, viscous=True)
    ro = sch(u, elements=els)
    kw = dict(dissipation=True, viscous=True, heat_flux=True, mu=1.0 / 1600, Pr=0.71, R=1.0)
    for prec, tol, what in ((sbp.FP64, TOL64, "NS FP64"), (sbp.FP32, TOL32, "NS FP32")):
        mesh = sbp.Mesh(desc, 3, precision=prec, **kw)
        _tuned(mesh, ud)
        r = mesh.residual(ud)
        mesh.check_device()
        _check_sampled(r.cpu().double().numpy(), ro, sch, u, els, tol, what)
        mesh.close()


def test_batch48_sampled():
    """The 48-problem batch (p ~ U{1..4}, n_e ~ logU[256, 16384], seed 0;
    190202 triangles in one persistent launch per call), tuned as the
    benchmark does: the residual on sampled elements of one problem of each
    degree and of the largest one, the VJP on two elements of each, and the
    finite-difference check of the whole batch (lambda ~ N(0,1), step 1e-6)."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.jacobian import vjp_elements
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[full batch48]")
    specs = wl.batch_problem_specs(48, 0)
    desc, deg, off = wl.batch_mesh(specs)
    meshes, states = [], []
    for b, sp in enumerate(specs):
        m = OracleMesh(wl.sub_mesh(desc, off[b], off[b + 1]), sp["p"])
        meshes.append(m)
        states.append(state(m, "batch", seed=1000 + b))
    lams = [np.random.default_rng(2000 + b).standard_normal(s.shape) for b, s in enumerate(states)]
    dirs = [np.random.default_rng(3000 + b).standard_normal(s.shape) * np.abs(s) for b, s in enumerate(states)]
    mesh = sbp.Mesh(desc, deg, problem_off=off)
    nc = int(mesh.n_c)
    lo = [int(mesh.node_off[off[b]]) * nc for b in range(len(specs) + 1)]
    assert all(lo[b + 1] - lo[b] == states[b].size for b in range(len(specs)))   # no padding

    def flat(parts):          # elements of one problem are contiguous, one n_p each
        out = np.zeros(int(mesh.n_nodes) * nc)
        for b, a in enumerate(parts):
            out[lo[b]:lo[b + 1]] = a.ravel()
        return torch.from_numpy(out).cuda()

    def part(x, b):
        return x[lo[b]:lo[b + 1]].reshape(states[b].shape)

    u, lam, v = flat(states), flat(lams), flat(dirs)
    _tuned(mesh, u, lam)
    r = mesh.residual(u).cpu().numpy()
    ub = mesh.vjp(u, lam).cpu().numpy()
    mesh.check_device()
    pick = sorted({[s["p"] for s in specs].index(q) for q in (1, 2, 3, 4)}
                  | {int(np.argmax([m.ne for m in meshes]))})
    for b in pick:
        m = meshes[b]
        sch = OracleScheme(m, ph.Gas())
        els = _sample(m.ne, 8, 500 + b)
        ro = sch(states[b], elements=els)
        _check_sampled(part(r, b), ro, sch, states[b], els, TOL64, f"problem {b} p={specs[b]['p']} ne={m.ne}")
        vel = els[:2]
        ref = vjp_elements(sch, states[b], lams[b], vel)
        sc = max(np.abs(ref[e]).max() for e in vel)
        err = max(np.abs(part(ub, b)[e] - ref[e]).max() for e in vel) / sc
        say(f"   problem {b}: VJP rel err {err:.2e}")
        assert err <= TOL64, (b, err)
    h = 1e-6
    fd = float(torch.sum(lam * (mesh.residual(u + h * v) - mesh.residual(u - h * v))) / (2 * h))
    ad = float(torch.sum(v * torch.from_numpy(ub).cuda()))
    say(f"   FD {fd:.12e} VJP {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}")
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    mesh.check_device()
    mesh.close()
