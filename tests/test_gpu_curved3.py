"""Entropy split on tetrahedra with quadratic maps (Assumption 1: p >= 2)
against the oracle: residual and entropy rate (FP64, ± dissipation), FP32,
free stream, sampled elements of the paper's 3D vortex grid, relaxation RK4
steps, the 3D vortex of the accuracy study with the studies' error norm,
and the refusals of the paths this geometry does not cover."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state, term_scale

pytestmark = pytest.mark.gpu


def _setup(p, diss, precision=0, desc=None):
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    desc = wl.curved_tet_mesh(2, 1.0, 0.03) if desc is None else desc
    m = OracleMesh(desc, p)
    sch = OracleScheme(m, ph.Gas(), dissipation=diss)
    mesh = sbp.Mesh(desc, p, dissipation=diss, precision=precision)
    return m, sch, mesh


@pytest.mark.parametrize("p,diss", [(2, False), (2, True), (3, False), (3, True)])
def test_curved_tets_vs_oracle(p, diss):
    import torch
    from oracle import physics as ph
    say(f"[curved3] p={p} diss={diss}")
    m, sch, mesh = _setup(p, diss)
    u = state(m, "random", seed=40 + p, jitter=0.01)
    r, er = mesh.residual(torch.from_numpy(u).cuda(), entropy_rate=True)
    mesh.check_device()
    ro = sch(u)
    err = rel_err_per_component(r.cpu().numpy(), ro)
    say("   rel err per component", err.max())
    assert (err <= 1e-12).all(), err
    rate_o = sch.entropy_rate(u, ro)
    scale = sum(np.sum(m.geometry(e)["H"][None, :] * np.abs(ph.entropy_vars(u[e], sch.gas) * ro[e]))
                for e in range(m.ne))
    assert abs(float(er.cpu()[0]) - rate_o) <= 1e-12 * scale
    if not diss:
        assert abs(float(er.cpu()[0])) <= 1e-12 * scale   # entropy conservative on curved elements
    mesh.close()


@pytest.mark.parametrize("p", [2, 3])
def test_curved_tets_fp32(p):
    import torch
    from paper_2305_07181_amd import sbp
    say(f"[curved3] FP32 p={p}")
    m, sch, mesh = _setup(p, True, precision=sbp.FP32)
    u = state(m, "random", seed=7, jitter=0.01)
    r = mesh.residual(torch.from_numpy(u).cuda()).cpu().numpy()
    err = rel_err_per_component(r, sch(u))
    say("   FP32 rel err", err.max())
    assert (err <= 2e-4).all(), err
    mesh.check_device()
    mesh.close()


def test_curved_tets_free_stream():
    """A uniform state has zero residual (discrete metric identities of the
    quadratic map at p >= 2), to the rounding of the summed terms."""
    import torch
    say("[curved3] free stream")
    for p in (2, 3):
        m, sch, mesh = _setup(p, True)
        u = np.zeros((m.ne, 5, m.n_p))
        u[:, 0], u[:, 1], u[:, 2], u[:, 3] = 1.2, 0.3, -0.2, 0.1
        u[:, 4] = 2.5 + 0.5 * (0.09 + 0.04 + 0.01) / 1.2
        r = mesh.residual(torch.from_numpy(u).cuda()).cpu().numpy()
        sc = term_scale(sch, u, range(m.ne))
        say(f"   p={p}: max |r| / term scale", (np.abs(r).max(axis=(0, 2)) / sc).max())
        assert (np.abs(r).max(axis=(0, 2)) <= 1e-13 * sc).all()
        mesh.close()


def test_paper_vortex3d_grid_sampled():
    """The paper's curved 3D vortex grid (6^3 x 6 tetrahedra, p = 3, eq. curve
    3d vortex) with a smooth state: sampled elements against the oracle."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[curved3] paper vortex grid, sampled")
    desc = wl.paper_vortex3d_mesh(6)
    m = OracleMesh(desc, 3)
    sch = OracleScheme(m, ph.Gas(), dissipation=True)
    u = state(m, "random", seed=12)
    mesh = sbp.Mesh(desc, 3, dissipation=True)
    r = mesh.residual(torch.from_numpy(u).cuda()).cpu().numpy()
    mesh.check_device()
    els = np.random.default_rng(3).choice(m.ne, 16, replace=False)
    ro = sch(u, elements=els)
    sc = term_scale(sch, u, els)
    err = np.abs(r[els] - ro).max(axis=(0, 2)) / sc
    say("   err / term scale", err.max(), " (plain rel:", rel_err_per_component(r[els], ro).max(), ")")
    assert (err <= 1e-12).all(), err
    mesh.close()


def test_curved_tets_rrk_steps():
    """Two relaxation RK4 steps on curved tetrahedra: the state follows the
    oracle's steps and the entropy is conserved per step."""
    import torch
    from oracle import rrk
    say("[curved3] RRK")
    m, sch, mesh = _setup(2, False)
    u = state(m, "random", seed=5, jitter=0.005)
    ud = torch.from_numpy(u).cuda()
    uo = u.copy()
    dt = 2e-3
    for step in range(2):
        rep = mesh.rrk_step(ud, dt=dt)
        uo, g, _, _ = rrk.rrk4_step(sch, uo, dt)
        ds = rep["entropy_after"] - rep["entropy_before"]
        say(f"   step {step}: gamma {rep['gamma']:.15f} oracle {g:.15f} entropy change {ds:.2e}")
        assert abs(ds) <= 64 * 2.2e-16 * abs(rep["entropy_before"])
    err = rel_err_per_component(ud.cpu().numpy(), uo)
    say("   state rel err", err.max())
    assert (err <= 1e-10).all(), err
    mesh.check_device()
    mesh.close()


def test_curved_tets_refusals():
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[curved3] refusals")
    desc = wl.curved_tet_mesh(2, 2.0, 0.03)
    with pytest.raises(sbp.SbpError) as ei:          # Assumption 1: p >= 2
        sbp.Mesh(desc, 1)
    assert ei.value.code == sbp.SBP_EINVAL
    with pytest.raises(sbp.SbpError) as ei:          # viscous terms: the entropy-split form only
        sbp.Mesh(desc, 2, viscous=True, mu=0.01, form=sbp.FORM_HADAMARD)
    assert ei.value.code == sbp.SBP_ENOTSUP


@pytest.mark.parametrize("p,diss", [(2, False), (3, True)])
def test_curved_tets_hadamard_and_hybrid(p, diss):
    """The Hadamard form on curved tetrahedra (metric average of the two
    nodes per pair) against the oracle, with local conservation; and the
    hybrid scheme with random per-element flags against the oracle's."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[curved3] Hadamard / hybrid p={p} diss={diss}")
    desc = wl.curved_tet_mesh(2, 1.0, 0.03)
    m = OracleMesh(desc, p)
    u = state(m, "random", seed=60 + p, jitter=0.01)
    ud = torch.from_numpy(u).cuda()
    mh = sbp.Mesh(desc, p, dissipation=diss, form=sbp.FORM_HADAMARD)
    rh = mh.residual(ud).cpu().numpy()
    mh.check_device()
    ro = OracleScheme(m, ph.Gas(), form="hadamard", dissipation=diss)(u)
    err = rel_err_per_component(rh, ro)
    say("   Hadamard rel err", err.max())
    assert (err <= 1e-12).all(), err
    if not diss:
        # global conservation: sum_k 1^T H_k r_k = 0 per component
        H = m.H_all()
        tot = np.einsum("en,ecn->c", H, rh)
        scale = np.einsum("en,ecn->c", H, np.abs(rh))
        assert (np.abs(tot) <= 1e-13 * scale).all(), tot / scale
    mh.close()
    flags = np.random.default_rng(p).integers(0, 2, m.ne).astype(np.uint8)
    ms = sbp.Mesh(desc, p, dissipation=diss)
    fd = torch.from_numpy(flags).cuda()
    ms.set_volume_form(fd)
    r, er = ms.residual(ud, entropy_rate=True)
    ms.check_device()
    sch = OracleScheme(m, ph.Gas(), form="hybrid", element_form=flags, dissipation=diss)
    ro = sch(u)
    err = rel_err_per_component(r.cpu().numpy(), ro)
    say("   hybrid rel err", err.max(), "flags", int(flags.sum()), "of", m.ne)
    assert (err <= 1e-12).all(), err
    rate_o = sch.entropy_rate(u, ro)
    scale = sum(np.sum(m.geometry(e)["H"][None, :] * np.abs(ph.entropy_vars(u[e], sch.gas) * ro[e]))
                for e in range(m.ne))
    assert abs(float(er.cpu()[0]) - rate_o) <= 1e-12 * scale
    ms.close()


@pytest.mark.parametrize("p,quadratic", [(1, False), (2, True), (3, True)])
def test_vortex3d_fields_and_error_norm(p, quadratic):
    """The 3D vortex of the accuracy study: its nodal fields, the studies'
    error norm on affine and curved tetrahedra against the oracle's, and no
    source term (the residual is the plain one)."""
    import torch
    from oracle import mms
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[curved3] vortex3d p={p} quadratic={quadratic}")
    desc = wl.paper_vortex3d_mesh(3, quadratic=quadratic)
    m = OracleMesh(desc, p)
    gas = ph.Gas()
    mesh = sbp.Mesh(desc, p)
    u_plain = None
    t = 0.4
    xs = np.moveaxis(m.node_coords(), 1, 0)
    ue = np.ascontiguousarray(np.moveaxis(mms.vortex3d_state(xs, t, gas), 0, 1))
    up = np.ascontiguousarray(ue * (1.0 + 0.01 * np.random.default_rng(p).standard_normal(ue.shape)))
    ud = torch.from_numpy(up).cuda()
    u_plain = mesh.residual(ud).cpu().numpy()
    mesh.set_source(sbp.SOURCE_VORTEX3D)
    ug = mesh.source_state(t).cpu().numpy().reshape(ue.shape)
    assert (rel_err_per_component(ug[:, [0, 1, 2, 4]], ue[:, [0, 1, 2, 4]]) <= 1e-14).all()
    assert np.abs(ug[:, 3]).max() == 0.0
    assert np.array_equal(mesh.residual(ud).cpu().numpy(), u_plain)
    exact = lambda x: mms.vortex3d_state(x, t, gas)
    for uu in (up, ue):
        e = mesh.source_error(torch.from_numpy(uu).cuda(), t)
        eo = mms.l2_error_quadrature(uu, m, exact)
        say(f"   quadrature norm gpu {e.sum():.6e} oracle {eo.sum():.6e}")
        assert np.abs(e - eo).max() <= 1e-12 * np.abs(eo).max(), (e, eo)
    mesh.check_device()
    mesh.close()


def test_vortex3d_study_runs():
    """A short run of the vortex study on a coarse grid: entropy conserved
    without dissipation, removed with it, errors finite."""
    from paper_2305_07181_amd import studies
    say("[curved3] vortex3d study, coarse")
    for diss in (False, True):
        r = studies.vortex3d_run(4, 2, diss, tf=0.2)
        say("  ", r)
        assert r["t"] >= 0.2 and 0 < r["l2_error"] < 10.0
        if diss:
            assert r["entropy_change"] < 0
        else:
            assert abs(r["entropy_change"]) < 1e-12
