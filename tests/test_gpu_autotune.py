"""Launch shapes and the autotuner.  Every launch shape of a kernel slot
(kernel variant x persistent grid) must give the same residual and VJP as the
built-in shape, which is checked against the oracle on sampled elements; the
tuner reports the shapes it timed, keeps the fastest, and a second handle of
the same workload starts from that choice."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state, term_scale

pytestmark = pytest.mark.gpu

GRIDS = (1, 2, 0)


def _setup(dim, p, n, precision, seed):
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import workloads as wl
    desc = wl.periodic_tet_mesh(n, 1.0) if dim == 3 else wl.vortex2d_mesh(n, warp=0.05)
    m = OracleMesh(desc, p)
    u = state(m, "random", seed=seed, jitter=0.01)
    return desc, m, u


# enough elements that one resident set of workgroups does not cover every
# tile (grid 1 and 2 differ from one workgroup per tile)
@pytest.mark.parametrize("dim,p,n,prec", [(3, 3, 8, 0), (3, 2, 12, 1), (3, 1, 12, 0), (2, 4, 64, 0),
                                          (2, 1, 64, 0), (2, 2, 48, 1), (2, 3, 48, 0), (2, 4, 40, 1)])
def test_every_residual_launch_shape(dim, p, n, prec):
    import torch
    from oracle import physics as ph
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[shapes residual] dim={dim} p={p} n={n} precision={prec}")
    desc, m, u = _setup(dim, p, n, prec, seed=40 + p)
    mesh = sbp.Mesh(desc, p, dissipation=True, precision=prec)
    ud = torch.from_numpy(u).cuda()
    assert mesh.launch_shape("residual", p) == (0, 1)
    r0, e0 = mesh.residual(ud, entropy_rate=True)
    r0 = r0.cpu().double().numpy()
    e0 = float(e0.cpu()[0])
    els = [0, 1, m.ne // 2, m.ne - 1]
    sch = OracleScheme(m, ph.Gas(), dissipation=True)
    ro = sch(u, elements=els)
    if prec == 0:
        def vs_oracle(r):
            return rel_err_per_component(r[els], ro)
    else:
        # FP32: the error against the scale of the summed terms (the 1%
        # jitter makes the residual ~1/100 of its terms on the finer grids)
        sc = term_scale(sch, u, els)

        def vs_oracle(r):
            return np.abs(r[els] - ro).max(axis=(0, 2)) / sc
    err = vs_oracle(r0)
    say("   built-in shape vs oracle", err.max())
    tol = 1e-12 if prec == 0 else 1e-5
    assert (err <= tol).all(), err
    # 2D: two or one node rows per lane with the facet SATs before the pair
    # sums, or two rows with the SATs after them; 3D: skew operators in LDS
    # or via the caches
    nvar = 3 if dim == 2 else 2
    for v in range(nvar):
        for g in GRIDS:
            mesh.set_launch_shape("residual", p, v, g)
            assert mesh.launch_shape("residual", p) == (v, g)
            r, e = mesh.residual(ud, entropy_rate=True)
            mesh.check_device()
            r = r.cpu().double().numpy()
            if prec == 0:
                d = np.abs(r - r0).max() / np.abs(r0).max()
            else:
                # FP32 kernels of different operation order: against the
                # summed-term scale, as for the oracle comparison
                d = (np.abs(r[els] - r0[els]).max(axis=(0, 2)) / sc).max()
            de = abs(float(e.cpu()[0]) - e0) / abs(e0)
            eo = vs_oracle(r).max()
            say(f"   variant {v} grid {g}: vs oracle {eo:.1e}, vs built-in {d:.1e}, entropy rate {de:.1e}")
            # the grid only changes which workgroup runs a tile (bitwise equal
            # residual); the variants are different kernels of the same sums
            # (FMA contraction may differ): rounding-level agreement, for FP32
            # up to 1e-5 of max |r| over 25-60 accumulated products
            assert d <= (0.0 if v == 0 else (1e-13 if prec == 0 else 1e-5)), (v, g, d)
            assert eo <= tol, (v, g, eo)
            # FP32: the dissipative rate of the 1%-jittered state is a small
            # difference of single-precision residual values
            assert de <= (1e-11 if v == 0 or prec == 0 else 1e-4), (v, g, de)
    with pytest.raises(sbp.SbpError):
        mesh.set_launch_shape("residual", p, nvar, 1)
    with pytest.raises(sbp.SbpError):
        mesh.set_launch_shape("residual", p + 1 if p < 3 else 1 if dim == 2 else 2, 0, 1)
    mesh.close()


@pytest.mark.parametrize("dim,p,n", [(3, 2, 12), (3, 3, 4), (2, 3, 64)])
def test_every_vjp_launch_shape(dim, p, n):
    import torch
    from oracle import physics as ph
    from oracle.jacobian import vjp_elements
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[shapes vjp] dim={dim} p={p} n={n}")
    desc, m, u = _setup(dim, p, n, 0, seed=50 + p)
    lam = np.random.default_rng(5000 + p).standard_normal(u.shape)
    mesh = sbp.Mesh(desc, p, dissipation=True)
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    b0 = mesh.vjp(ud, ld).cpu().numpy()
    els = [0, m.ne - 1]
    ref = vjp_elements(OracleScheme(m, ph.Gas(), dissipation=True), u, lam, els)
    scale = max(np.abs(ref[e]).max() for e in els)
    err = max(np.abs(b0[e] - ref[e]).max() for e in els) / scale
    say("   built-in shape vs oracle", err)
    assert err <= 1e-12, err
    for v in (0, 1):
        for g in GRIDS:
            mesh.set_launch_shape("vjp", p, v, g)
            b = mesh.vjp(ud, ld).cpu().numpy()
            mesh.check_device()
            d = np.abs(b - b0).max() / np.abs(b0).max()
            say(f"   variant {v} grid {g}: diff {d:.1e}")
            assert d <= 1e-13, (v, g, d)
    mesh.close()


def test_autotune_keeps_a_timed_shape_and_remembers_it():
    import torch
    from paper_2305_07181_amd import sbp
    say("[autotune] 3D p=2, 10368 tetrahedra")
    desc, m, u = _setup(3, 2, 12, 0, seed=61)
    lam = np.random.default_rng(61).standard_normal(u.shape)
    mesh = sbp.Mesh(desc, 2, dissipation=True)
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    r0 = mesh.residual(ud).cpu().numpy()
    rep = mesh.autotune(ud, ld)
    say("  ", rep)
    assert [(t["kind"], t["p"]) for t in rep] == [("residual", 2), ("vjp", 2)]
    for t in rep:
        assert t["n_candidates"] == 6
        assert 0 < t["ms_best"] <= t["ms_builtin"]
        assert mesh.launch_shape(t["kind"], t["p"]) == (t["variant"], t["grid"])
    r1 = mesh.residual(ud).cpu().numpy()
    assert np.abs(r1 - r0).max() <= 1e-15 * np.abs(r0).max()
    # a new handle of the same workload starts from the tuned shapes
    other = sbp.Mesh(desc, 2, dissipation=True)
    for t in rep:
        assert other.launch_shape(t["kind"], t["p"]) == (t["variant"], t["grid"])
    other.close()
    # the RRK step re-captures its stage graph with the tuned shapes
    w = ud.clone()
    info = mesh.rrk_step(w, cfl=0.1)
    mesh.check_device()
    assert abs(info["entropy_after"] - info["entropy_before"] - info["gamma"] * info["e"]) <= \
        1e-12 * abs(info["entropy_before"])
    mesh.close()


def test_autotune_batched_2d():
    """A 2D mesh with several degrees has one batched launch per operation:
    the tuner times its three grids."""
    import torch
    from paper_2305_07181_amd import sbp
    from tests.test_gpu_batch import _batch, _flat
    say("[autotune] batched 2D")
    specs = [dict(p=1, nx=12, ny=10), dict(p=2, nx=10, ny=9), dict(p=3, nx=8, ny=8), dict(p=4, nx=7, ny=6)]
    desc, deg, off, meshes, states = _batch(specs, 0.05)
    mesh = sbp.Mesh(desc, deg, dissipation=False, problem_off=off)
    ud = torch.from_numpy(_flat(mesh, off, states)).cuda()
    lam = torch.from_numpy(np.random.default_rng(71).standard_normal(ud.numel())).cuda()
    r0 = mesh.residual(ud).cpu()
    b0 = mesh.vjp(ud, lam).cpu()
    rep = mesh.autotune(ud, lam)
    say("  ", rep)
    assert [(t["kind"], t["p"]) for t in rep] == [("residual", 0), ("vjp", 0)]
    for t in rep:
        assert t["n_candidates"] == 3 and t["variant"] == 0
        assert mesh.launch_shape(t["kind"], 0) == (0, t["grid"])
    for g in GRIDS:
        mesh.set_launch_shape("residual", 0, 0, g)
        mesh.set_launch_shape("vjp", 0, 0, g)
        assert torch.equal(mesh.residual(ud).cpu(), r0), g
        d = (mesh.vjp(ud, lam).cpu() - b0).abs().max() / b0.abs().max()
        assert d <= 1e-13, (g, float(d))
    mesh.check_device()
    mesh.close()
