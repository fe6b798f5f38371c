"""GPU parity of the HIP residual against the CPU oracle (through the C ABI).

Tolerances:
  * FP64: max_nodes |r_gpu - r_orc|_c <= 1e-12 max_nodes |r_orc|_c per
    conserved variable; for the low-Mach Taylor-Green state the denominator
    is the magnitude of the summed terms (the residual is ~1e-2 of them).
  * FP32: the same measure <= 2e-4 (single precision, n_p-term sums).
"""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state, term_scale

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu_residual(desc, p, u, **kw):
    torch = _torch()
    from paper_2305_07181_amd import sbp
    mesh = sbp.Mesh(desc, p, **kw)
    ud = torch.from_numpy(u).cuda()
    r, er = mesh.residual(ud, entropy_rate=True)
    torch.cuda.synchronize()
    mesh.check_device()
    out = r.cpu().double().numpy(), float(er.cpu()[0])
    mesh.close()
    return out


def _oracle(desc, p, **kw):
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    m = OracleMesh(desc, p)
    return m, OracleScheme(m, ph.Gas(), **kw)


CASES_2D = [(p, warp, diss) for p in (1, 2, 3, 4) for warp in (0.0, 0.05) for diss in (False, True)]


@pytest.mark.parametrize("p,warp,diss", CASES_2D)
def test_parity_2d_triangles(p, warp, diss):
    """Small curved/affine periodic triangle meshes (several tiles plus a
    ragged last tile), discontinuous random state."""
    from paper_2305_07181_amd import workloads as wl
    say(f"[2d] p={p} warp={warp} diss={diss}")
    desc = wl.periodic_tri_mesh(5, 4, 20.0, 16.0) if warp == 0.0 else wl.vortex2d_mesh(5, warp=warp)
    m, sch = _oracle(desc, p, dissipation=diss)
    u = state(m, "random", seed=11, jitter=0.01)
    r_gpu, er_gpu = _gpu_residual(desc, p, u, dissipation=diss)
    r_orc = sch(u)
    err = rel_err_per_component(r_gpu, r_orc)
    say("   rel err per component", err)
    assert (err <= TOL64).all(), err
    er_orc = sch.entropy_rate(u, r_orc)
    scale = np.sum(np.abs(r_orc)) * 10
    assert abs(er_gpu - er_orc) <= 1e-12 * scale
    if not diss:
        assert abs(er_gpu) <= 1e-12 * scale


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("diss", [False, True])
def test_parity_3d_tetrahedra(p, diss):
    from paper_2305_07181_amd import workloads as wl
    say(f"[3d] p={p} diss={diss}")
    desc = wl.periodic_tet_mesh(2, 1.0)          # 48 tets
    m, sch = _oracle(desc, p, dissipation=diss)
    u = state(m, "random", seed=5, jitter=0.01)
    r_gpu, er_gpu = _gpu_residual(desc, p, u, dissipation=diss)
    r_orc = sch(u)
    err = rel_err_per_component(r_gpu, r_orc)
    say("   rel err per component", err)
    assert (err <= TOL64).all(), err


def test_parity_vortex_128_triangles():
    """The 128-triangle p=2 vortex (EC SATs, no dissipation)."""
    from paper_2305_07181_amd import workloads as wl
    say("[vortex128]")
    desc = wl.vortex2d_mesh(8)
    m, sch = _oracle(desc, 2)
    u = state(m, "vortex")
    r_gpu, er_gpu = _gpu_residual(desc, 2, u)
    r_orc = sch(u)
    err = rel_err_per_component(r_gpu, r_orc)
    say("   rel err per component", err, "entropy rate", er_gpu)
    assert (err <= TOL64).all(), err
    assert abs(er_gpu) < 1e-13 * np.abs(r_orc).sum()


@pytest.mark.parametrize("p", [2, 3])
def test_parity_taylor_green_small(p):
    """Low-Mach TGV on 3^3 x 6 tets with dissipation: tolerance against the
    scale of the summed terms (the residual is a small difference of them)."""
    from paper_2305_07181_amd import workloads as wl
    say(f"[tgv small] p={p}")
    desc = wl.tgv_mesh(3)
    m, sch = _oracle(desc, p, dissipation=True)
    u = state(m, "tgv")
    r_gpu, _ = _gpu_residual(desc, p, u, dissipation=True)
    r_orc = sch(u)
    els = list(range(m.ne))
    sc = term_scale(sch, u, els)
    err = np.abs(r_gpu - r_orc).max(axis=(0, 2)) / sc
    say("   err / term scale", err, " (plain rel:", rel_err_per_component(r_gpu, r_orc), ")")
    assert (err <= TOL64).all(), err


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_parity_hadamard(dim, p):
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[hadamard] dim={dim} p={p}")
    desc = wl.vortex2d_mesh(4, warp=0.05) if dim == 2 else wl.periodic_tet_mesh(2, 1.0)
    m, sch = _oracle(desc, p, form="hadamard", dissipation=True)
    u = state(m, "random", seed=3, jitter=0.01)
    r_gpu, _ = _gpu_residual(desc, p, u, form=sbp.FORM_HADAMARD, dissipation=True)
    r_orc = sch(u)
    err = rel_err_per_component(r_gpu, r_orc)
    say("   rel err per component", err)
    assert (err <= TOL64).all(), err
    # local conservation of the Hadamard form: sum_k 1^T H_k r_k = 0
    H = m.H_all()
    tot = np.einsum("en,ecn->c", H, r_gpu)
    assert (np.abs(tot) <= 1e-12 * np.einsum("en,ecn->c", H, np.abs(r_gpu))).all()


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_fp32_error_vs_fp64_oracle(dim, p):
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[fp32] dim={dim} p={p}")
    desc = wl.vortex2d_mesh(4, warp=0.05) if dim == 2 else wl.periodic_tet_mesh(2, 1.0)
    m, sch = _oracle(desc, p, dissipation=True)
    u = state(m, "random", seed=9, jitter=0.01)
    r_gpu, _ = _gpu_residual(desc, p, u, dissipation=True, precision=sbp.FP32)
    r_orc = sch(u)
    err = rel_err_per_component(r_gpu, r_orc)
    say("   FP32 rel err per component", err)
    assert (err <= 2e-4).all(), err


def test_nonphysical_state_is_reported():
    torch = _torch()
    from paper_2305_07181_amd import sbp, workloads as wl
    from oracle.geometry import OracleMesh
    say("[nonphys]")
    desc = wl.vortex2d_mesh(2)
    m = OracleMesh(desc, 1)
    u = state(m, "vortex")
    u[3, 3, 2] = 0.0      # energy 0 -> negative pressure at one node
    mesh = sbp.Mesh(desc, 1)
    ud = torch.from_numpy(u).cuda()
    mesh.residual(ud)
    with pytest.raises(sbp.SbpError) as ei:
        mesh.check_device()
    assert ei.value.code == sbp.SBP_ENONPHYS
    mesh.check_device()   # flag cleared


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("heat", [True, False])
def test_parity_navier_stokes_3d(p, heat):
    """Navier-Stokes terms with Baumann-Oden SATs (Sec. 5) plus matrix
    dissipation on 48 tets; without heat flux the entropy rate is <= 0."""
    torch = _torch()
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say(f"[ns3d] p={p} heat={heat}")
    desc = wl.periodic_tet_mesh(2, 1.0)
    m = OracleMesh(desc, p)
    gas = ph.Gas(mu=0.05, Pr=0.71, R=1.0, heat_flux=heat)
    sch = OracleScheme(m, gas, dissipation=True, viscous=True)
    u = state(m, "random", seed=4, jitter=0.01)
    mesh = sbp.Mesh(desc, p, dissipation=True, viscous=True, heat_flux=heat, mu=0.05, Pr=0.71, R=1.0)
    ud = torch.from_numpy(u).cuda()
    r, er = mesh.residual(ud, entropy_rate=True)
    r = r.cpu().numpy()
    mesh.check_device()
    ro = sch(u)
    err = rel_err_per_component(r, ro)
    say("   rel err per component", err, "entropy rate", float(er.cpu()[0]))
    assert (err <= TOL64).all(), err
    if not heat:
        assert float(er.cpu()[0]) < 0
    mesh.close()


def test_parity_navier_stokes_tgv_fp32():
    """FP32 Navier-Stokes residual on the low-Mach TGV (Re = 1600, heat flux
    on) against the FP64 oracle, scaled by the summed-term magnitude."""
    torch = _torch()
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[ns tgv fp32]")
    desc = wl.tgv_mesh(3)
    m = OracleMesh(desc, 3)
    gas = ph.Gas(mu=1.0 / 1600, Pr=0.71, R=1.0)
    sch = OracleScheme(m, gas, dissipation=True, viscous=True)
    u = state(m, "tgv")
    for prec, tol in ((sbp.FP64, TOL64), (sbp.FP32, 2e-6)):
        mesh = sbp.Mesh(desc, 3, dissipation=True, viscous=True, mu=1.0 / 1600, precision=prec)
        r = mesh.residual(torch.from_numpy(u).cuda()).cpu().double().numpy()
        mesh.close()
        ro = sch(u)
        sc = term_scale(sch, u, list(range(m.ne)))
        err = np.abs(r - ro).max(axis=(0, 2)) / sc
        say("   precision", prec, "err / term scale", err)
        assert (err <= tol).all(), err
