"""Navier-Stokes terms (Sec. 5: viscous flux with heat flux, Baumann-Oden
SATs, eq. bo sats) on triangles (affine and with quadratic maps) and on
tetrahedra with quadratic maps, against the oracle's dense-operator
residual: FP64 at 1e-12 per conserved variable (jittered random states, so
both exponential-average branches and nonzero interface jumps enter), the
FP64 entropy rate, its sign without heat flux (viscous terms dissipate),
FP32 against the summed-term scale, and free-stream preservation."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state, term_scale

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

CASES = ([("tri", p, h, d) for p in (1, 2, 3, 4) for h, d in ((True, False), (False, True))]
         + [("tri-curved", p, h, d) for p in (1, 2, 3, 4) for h, d in ((True, True), (False, False))]
         + [("tet-curved", p, h, d) for p in (2, 3) for h, d in ((True, False), (False, True))])


def _desc(kind):
    from paper_2305_07181_amd import workloads as wl
    if kind == "tri":
        return wl.vortex2d_mesh(4)
    if kind == "tri-curved":
        return wl.mms_mesh2d(4)
    return wl.mms_mesh3d(2, curve="quadratic")


@pytest.mark.parametrize("kind,p,heat,diss", CASES)
def test_parity_navier_stokes(kind, p, heat, diss):
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[ns] {kind} p={p} heat={heat} diss={diss}")
    desc = _desc(kind)
    m = OracleMesh(desc, p)
    gas = ph.Gas(mu=0.05, Pr=0.71, R=1.0, heat_flux=heat)
    sch = OracleScheme(m, gas, dissipation=diss, viscous=True)
    u = state(m, "random", seed=14 + p, jitter=0.01)
    mesh = sbp.Mesh(desc, p, dissipation=diss, viscous=True, heat_flux=heat, mu=0.05, Pr=0.71, R=1.0)
    ud = torch.from_numpy(u).cuda()
    r, er = mesh.residual(ud, entropy_rate=True)
    r = r.cpu().numpy()
    mesh.check_device()
    mesh.close()
    ro = sch(u)
    err = rel_err_per_component(r, ro)
    rate_o = sch.entropy_rate(u, ro)
    scale = sum(np.sum(m.geometry(e)["H"][None, :] * np.abs(ph.entropy_vars(u[e], gas) * ro[e]))
                for e in range(m.ne))
    say("   rel err per component", err, "entropy rate", float(er.cpu()[0]), "oracle", rate_o)
    assert (err <= TOL64).all(), err
    assert abs(float(er.cpu()[0]) - rate_o) <= 1e-12 * scale
    if not heat:
        assert float(er.cpu()[0]) < 0


@pytest.mark.parametrize("kind,p", [("tri-curved", 4), ("tet-curved", 3)])
def test_navier_stokes_fp32_and_free_stream(kind, p):
    """FP32 against the FP64 oracle over the summed-term scale; a uniform
    state gives a zero residual (free stream) on the curved grids."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[ns fp32 / free stream] {kind} p={p}")
    desc = _desc(kind)
    m = OracleMesh(desc, p)
    gas = ph.Gas(mu=0.05, Pr=0.71, R=1.0, heat_flux=True)
    sch = OracleScheme(m, gas, dissipation=True, viscous=True)
    u = state(m, "random", seed=24, jitter=0.01)
    kw = dict(dissipation=True, viscous=True, mu=0.05, Pr=0.71, R=1.0)
    mesh = sbp.Mesh(desc, p, precision=sbp.FP32, **kw)
    r = mesh.residual(torch.from_numpy(u).cuda()).cpu().double().numpy()
    mesh.check_device()
    mesh.close()
    els = list(range(m.ne))
    sc = term_scale(sch, u, els)
    err = np.abs(r - sch(u)).max(axis=(0, 2)) / sc
    say("   FP32 err / term scale", err)
    assert (err <= 1e-5).all(), err
    uf = np.array(u)
    rho, V, pr = 1.1, (0.3, -0.2, 0.1)[:m.dim], 0.9
    uf[:, 0] = rho
    for i in range(m.dim):
        uf[:, 1 + i] = rho * V[i]
    uf[:, m.dim + 1] = pr / 0.4 + 0.5 * rho * sum(v * v for v in V)
    mesh = sbp.Mesh(desc, p, **kw)
    r = mesh.residual(torch.from_numpy(uf).cuda()).cpu().numpy()
    mesh.close()
    say("   free stream max |r|", np.abs(r).max())
    assert np.abs(r).max() <= 1e-12
