"""GPU relaxation RK4 against the oracle's (Sec. 6.1): the 128-triangle p=2
isentropic vortex, EC SATs, CFL 0.1, 20 steps; and fully discrete entropy
conservation on the GPU."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state

pytestmark = pytest.mark.gpu


def test_rrk_vortex_20_steps_parity():
    """Per step: dt agrees to 1e-13 plus four times the states' relative
    difference after the previous step (dt = CFL min h / (|V| + a) moves with
    the state, relative sensitivity below 2); the GPU's gamma is a root of the oracle's
    r(gamma) within its rounding (|r(gamma_gpu)| <= 8 eps sum H|s|); gamma
    agrees within the root's conditioning kappa = 8 eps sum H|s| / |r'(gamma)|;
    the states agree within the accumulated bound sum_n (1e-12 + kappa_n
    max|d_n| / max|u|) (relative, per component); entropy is conserved to
    roundoff on the GPU."""
    import torch
    from oracle import physics as ph
    from oracle import rrk
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[rrk vortex 20 steps]")
    eps = np.finfo(float).eps
    desc = wl.vortex2d_mesh(8)
    m = OracleMesh(desc, 2)
    sch = OracleScheme(m, ph.Gas())
    u = state(m, "vortex")
    mesh = sbp.Mesh(desc, 2)
    ud = torch.from_numpy(u).cuda()
    s0 = sch.total_entropy(u)
    uo = u.copy()
    H = m.H_all()
    bound = 0.0
    err_prev = 0.0
    for step in range(20):
        dt_o = sch.timestep(uo, 0.1)
        rep = mesh.rrk_step(ud, cfl=0.1)
        assert abs(rep["dt"] - dt_o) <= (1e-13 + 4 * err_prev) * dt_o, (rep["dt"], dt_o, err_prev)
        d, e = rrk.rk4_direction(sch, uo, dt_o)
        g = rrk.solve_gamma(sch, uo, d, e)
        s_abs = np.sum(H * np.abs(ph.entropy(np.moveaxis(uo, 1, 0), sch.gas)))
        w1 = np.stack([ph.entropy_vars(uo[k] + g * d[k], sch.gas) for k in range(m.ne)])
        rprime = np.sum(H[:, None, :] * w1 * d) - e
        kappa = 8 * eps * s_abs / abs(rprime)
        r_at_gpu = rrk.entropy_gap(sch, uo, d, e, rep["gamma"], H)
        assert abs(r_at_gpu) <= 8 * eps * s_abs, (r_at_gpu, 8 * eps * s_abs)
        assert abs(rep["gamma"] - g) <= kappa
        uo = uo + g * d
        bound += 1e-12 + kappa * np.abs(d).max() / np.abs(uo).max()
        ug = ud.cpu().numpy()
        err = np.abs(ug - uo).max(axis=(0, 2)) / np.abs(uo).max(axis=(0, 2))
        ds = (rep["entropy_after"] - s0) / abs(s0)
        say(f"   step {step}: gamma gpu {rep['gamma']:.16f} oracle {g:.16f} (kappa {kappa:.1e}) | "
            f"rel err {err.max():.2e} (bound {bound:.1e}) | entropy change {ds:.2e} | iters {rep['iters']}")
        assert (err <= bound).all(), err
        assert abs(ds) <= 1e-13
        err_prev = float(err.max())
    mesh.close()


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2)])
def test_rrk_entropy_dissipation_and_conservation(dim, p):
    """With dissipation the step removes entropy by exactly gamma e; without,
    the total entropy is constant to roundoff (GPU FP64 sums)."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[rrk entropy] dim={dim} p={p}")
    desc = wl.vortex2d_mesh(4, warp=0.05) if dim == 2 else wl.periodic_tet_mesh(2, 1.0)
    m = OracleMesh(desc, p)
    u = state(m, "random", seed=2, jitter=0.01)
    for diss in (False, True):
        mesh = sbp.Mesh(desc, p, dissipation=diss)
        ud = torch.from_numpy(u).cuda()
        reps = [mesh.rrk_step(ud, cfl=0.1) for _ in range(3)]
        for rep in reps:
            ds = rep["entropy_after"] - rep["entropy_before"]
            scale = abs(rep["entropy_before"])
            assert abs(ds - rep["gamma"] * rep["e"]) <= 64 * 2.2e-16 * scale
            if diss:
                assert rep["e"] < 0
            else:
                assert abs(ds) <= 64 * 2.2e-16 * scale
        say("   diss", diss, "gammas", [r["gamma"] for r in reps])
        mesh.close()


@pytest.mark.parametrize("dim,p,prec", [(2, 4, 0), (3, 3, 1)])
def test_rrk_graph_replay_matches_eager(dim, p, prec):
    """The captured stage graph replayed over several steps (with eager
    residual calls in between) gives bit-identical states to launching the
    stages one by one."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[rrk graph] dim={dim} p={p} prec={prec}")
    desc = wl.vortex2d_mesh(6, warp=0.05) if dim == 2 else wl.tgv_mesh(3)
    m = OracleMesh(desc, p)
    u = state(m, "vortex" if dim == 2 else "tgv")
    kw = dict(dissipation=True, precision=prec)
    if dim == 3:
        kw.update(viscous=True, mu=1.0 / 1600)
    mg = sbp.Mesh(desc, p, **kw)
    me = sbp.Mesh(desc, p, **kw)
    me.use_graphs(False)
    ug = torch.from_numpy(u).cuda()
    ue = ug.clone()
    for step in range(5):
        rg = mg.rrk_step(ug, cfl=0.2)
        me.residual(ue)            # eager work between the replays
        re_ = me.rrk_step(ue, cfl=0.2)
        assert rg["gamma"] == re_["gamma"] and rg["dt"] == re_["dt"]
        assert torch.equal(ug, ue), float((ug - ue).abs().max())
        say(f"   step {step}: gamma {rg['gamma']:.15f} iters {rg['iters']} entropy change "
            f"{rg['entropy_after'] - rg['entropy_before']:.3e}")
        if dim == 3:
            assert rg["entropy_after"] <= rg["entropy_before"]
    mg.close()
    me.close()


def test_rrk_navier_stokes_tgv_first_steps_vs_oracle():
    """The first relaxation RK4 steps of the Navier-Stokes Taylor-Green run
    (3^3 x 6 tetrahedra, p = 3, Re = 1600, Pr = 0.71, heat flux and matrix
    dissipation, FP64, captured stage graph) against the oracle's steps: the
    GPU's gamma is a root of the oracle's r(gamma) within its rounding
    (|r| <= 8 eps sum H|s|) and agrees within the root's conditioning
    kappa = 8 eps sum H|s| / |r'(gamma)| (large here: at M = 0.1 the step
    changes the entropy by little against its size); the states agree within
    sum_n (1e-12 + kappa_n max|d_n,c| / max|u_c|) for each component c (the
    z momentum grows from zero, so its own scale is the one to use)."""
    import torch
    from oracle import physics as ph
    from oracle import rrk
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[rrk ns tgv] first steps vs oracle")
    eps = np.finfo(float).eps
    desc = wl.tgv_mesh(3)
    m = OracleMesh(desc, 3)
    gas = ph.Gas(mu=1.0 / 1600, Pr=0.71, R=1.0)
    sch = OracleScheme(m, gas, dissipation=True, viscous=True)
    H = m.H_all()
    u = state(m, "tgv")
    mesh = sbp.Mesh(desc, 3, dissipation=True, viscous=True, heat_flux=True, mu=1.0 / 1600, Pr=0.71, R=1.0)
    ud = torch.from_numpy(u).cuda()
    uo, to = u.copy(), 0.0
    dt = sch.timestep(u, 0.2)
    bound = 0.0
    for step in range(3):
        rep = mesh.rrk_step(ud, dt=dt)
        d, e = rrk.rk4_direction(sch, uo, dt)
        g = rrk.solve_gamma(sch, uo, d, e)
        s_abs = np.sum(H * np.abs(ph.entropy(np.moveaxis(uo, 1, 0), gas)))
        w1 = np.stack([ph.entropy_vars(uo[k] + g * d[k], gas) for k in range(m.ne)])
        kappa = 8 * eps * s_abs / abs(np.sum(H[:, None, :] * w1 * d) - e)
        r_at_gpu = rrk.entropy_gap(sch, uo, d, e, rep["gamma"], H)
        say(f"   step {step}: gamma gpu {rep['gamma']:.15f} oracle {g:.15f} (kappa {kappa:.1e})")
        assert abs(r_at_gpu) <= 8 * eps * s_abs, (r_at_gpu, 8 * eps * s_abs)
        assert abs(rep["gamma"] - g) <= kappa
        uo = uo + g * d
        to += g * dt
        assert abs(rep["t"] - to) <= kappa * dt + 1e-15
        bound = bound + 1e-12 + kappa * np.abs(d).max(axis=(0, 2)) / np.abs(uo).max(axis=(0, 2))
    err = rel_err_per_component(ud.cpu().numpy(), uo)
    say("   state rel err", err, "bound", bound)
    assert (err <= bound).all(), (err, bound)
    mesh.check_device()
    mesh.close()


@pytest.mark.parametrize("viscous", [False, True])
def test_rrk_report_entropies_3d(viscous):
    """The step's report in 3D (n_c + 2 = 7 diagnostics exist; the step
    reduces only the total entropy): entropy_before and entropy_after are
    bitwise the total entropy sbp_diagnostics gives before and after."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[rrk report 3d] viscous={viscous}")
    desc = wl.tgv_mesh(2)
    m = OracleMesh(desc, 2)
    ud = torch.from_numpy(state(m, "tgv")).cuda()
    kw = dict(viscous=True, mu=1.0 / 1600) if viscous else {}
    mesh = sbp.Mesh(desc, 2, dissipation=True, **kw)
    for _ in range(2):
        d0 = mesh.diagnostics(ud)
        rep = mesh.rrk_step(ud, cfl=0.1)
        d1 = mesh.diagnostics(ud)
        assert len(d0) == 7
        assert rep["entropy_before"] == d0[0] and rep["entropy_after"] == d1[0]
        assert rep["entropy_after"] <= rep["entropy_before"]
    mesh.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_rrk_without_report_same_state(graphs):
    """sbp_rrk_step with a null report (a second captured sequence, without the
    entropy sums) advances u bit-identically to the step with a report."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[rrk no report] graphs={graphs}")
    desc = wl.vortex2d_mesh(6, warp=0.05)
    m = OracleMesh(desc, 3)
    u = torch.from_numpy(state(m, "vortex")).cuda()
    ma = sbp.Mesh(desc, 3, dissipation=True)
    mb = sbp.Mesh(desc, 3, dissipation=True)
    ma.use_graphs(graphs)
    mb.use_graphs(graphs)
    ua, ub = u.clone(), u.clone()
    for _ in range(3):
        rep = ma.rrk_step(ua, cfl=0.2)
        assert mb.rrk_step(ub, cfl=0.2, report=False) is None
        assert torch.equal(ua, ub)
        assert rep["iters"] >= 1 and 0.5 < rep["gamma"] < 1.5
    ma.close()
    mb.close()


def test_rrk_nonphysical_state_leaves_u_unchanged():
    """A state with negative pressure at one node: the step returns
    SBP_ENONPHYS and u keeps its bytes (the device update is skipped when a
    kernel of the step has flagged the state)."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[rrk nonphys]")
    desc = wl.vortex2d_mesh(4)
    m = OracleMesh(desc, 2)
    u = state(m, "vortex")
    u[5, 3, 1] = 0.0                       # energy 0 -> negative pressure
    mesh = sbp.Mesh(desc, 2, dissipation=True)
    ud = torch.from_numpy(u).cuda()
    u0 = ud.clone()
    with pytest.raises(sbp.SbpError) as ei:
        mesh.rrk_step(ud, dt=1e-3)
    assert ei.value.code == sbp.SBP_ENONPHYS
    assert torch.equal(ud, u0)
    mesh.check_device()                    # flag cleared
    mesh.close()
