"""The primary-conservation study (Sec. 4.3, Thm. conservation) through the
library on small grids: the conserved sums it reports are the oracle's sums
of the same states, the relaxation step keeps the entropy, and the errors
fall with refinement; the kinetic energy of the diagnostics and the
Taylor-Green history (Sec. 7.5)."""
import numpy as np
import pytest

from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def test_conserved_sums_match_oracle():
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[study] conserved sums")
    desc = wl.paper_vortex2d_mesh(8)
    m = OracleMesh(desc, 2)
    x = m.node_coords()
    rho, V, pr = wl.paper_vortex2d(np.moveaxis(x, 1, 0))
    u = np.ascontiguousarray(np.moveaxis(wl.conservative(rho, V, pr), 0, 1))
    mesh = sbp.Mesh(desc, 2)
    ud = torch.from_numpy(u).cuda()
    for _ in range(3):
        mesh.rrk_step(ud, cfl=0.1)
    d = mesh.diagnostics(ud)
    mesh.check_device()
    uf = ud.cpu().numpy()
    H = m.H_all()
    sums = np.einsum("en,ecn->c", H, uf)
    s_o = sum(np.sum(H[e] * ph.entropy(uf[e], ph.Gas())) for e in range(m.ne))
    say("   gpu", d, "oracle", s_o, sums)
    assert abs(d[0] - s_o) <= 1e-13 * abs(s_o)
    assert np.allclose(d[1:1 + m.n_c], sums, rtol=1e-13, atol=1e-13 * np.abs(sums).max())
    mesh.close()


def test_conservation_study_small():
    from paper_2305_07181_amd import studies
    say("[study] small grids")
    rows = studies.conservation_study([8, 16], [2], tf=0.5, cfl=0.1, emit=say)
    for r in rows:
        assert abs(r["entropy_change"]) < 1e-12          # entropy conservative + relaxation
        assert 0 < r["mass_error"] < 1e-2 and 0 < r["energy_error"] < 1e-2
        assert r["t"] >= 0.5
    assert rows[1]["mass_error"] < rows[0]["mass_error"]


@pytest.mark.parametrize("dim,p,ns", [(2, 2, (8, 16)), (3, 1, (4, 8)), (3, 2, (3, 6))])
def test_mms_study_small(dim, p, ns):
    """Manufactured solution (Sec. 7) through the library on two small grids:
    the nodal fields start exact; after 50 steps to t = 10^-3 the studies'
    error (degree 3p+1 rule) falls at about p + 1 (the fit of the element
    polynomials dominates this early) and the nodal error at least at the
    truncation order p (t times the truncation error)."""
    from paper_2305_07181_amd import studies
    say(f"[study] mms dim={dim} p={p}")
    rows = studies.mms_study(dim, ns, [p], tf=1e-3, steps=50, emit=say)
    for r in rows:
        assert r["initial_error_nodal"] < 1e-13
        assert abs(r["t"] - 1e-3) < 1e-9
        assert 0 < r["l2_error"] < 1.0 and 0 < r["l2_error_nodal"] < 1e-2
    assert rows[1]["rate"] > p + 0.5, rows[1]["rate"]
    assert rows[1]["rate_nodal"] > p - 0.35, rows[1]["rate_nodal"]


def test_vortex2d_fields_and_error_norm():
    """The 2D vortex of the accuracy study: nodal fields against the input
    generator's, the studies' error norm against the oracle's on the curved
    grid, no source term."""
    import torch
    from oracle import mms
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[study] vortex2d fields and norm")
    desc = wl.paper_vortex2d_mesh(8)
    for p in (1, 4):
        m = OracleMesh(desc, p)
        gas = ph.Gas()
        t = 0.7
        exact = lambda x: _cons(*wl.paper_vortex2d(x, t))
        xs = np.moveaxis(m.node_coords(), 1, 0)
        ue = np.ascontiguousarray(np.moveaxis(exact(xs), 0, 1))
        mesh = sbp.Mesh(desc, p)
        up = np.ascontiguousarray(ue * (1.0 + 0.01 * np.random.default_rng(p).standard_normal(ue.shape)))
        ud = torch.from_numpy(up).cuda()
        r0 = mesh.residual(ud).cpu().numpy()
        mesh.set_source(sbp.SOURCE_VORTEX2D)
        ug = mesh.source_state(t).cpu().numpy().reshape(ue.shape)
        err = np.abs(ug - ue).max(axis=(0, 2)) / np.abs(ue).max(axis=(0, 2))
        assert (err <= 1e-14).all(), err
        assert np.array_equal(mesh.residual(ud).cpu().numpy(), r0)
        for uu in (up, ue):
            e = mesh.source_error(torch.from_numpy(uu).cuda(), t)
            eo = mms.l2_error_quadrature(uu, m, exact)
            say(f"   p={p} quadrature norm gpu {e.sum():.6e} oracle {eo.sum():.6e}")
            assert np.abs(e - eo).max() <= 1e-12 * np.abs(eo).max(), (e, eo)
        mesh.check_device()
        mesh.close()


def _cons(rho, V, p):
    from paper_2305_07181_amd import workloads as wl
    return wl.conservative(rho, V, p)


@pytest.mark.parametrize("p", [2, 3])
def test_vortex2d_rates_small(p):
    """The 2D vortex on two grids (20^2 x 2, 40^2 x 2) to t = 0.5: the
    error in the studies' norm falls at a rate in [p - 0.2, p + 1.2], the
    accuracy pin for the entropy-conservative scheme."""
    from paper_2305_07181_amd import studies
    say(f"[study] vortex2d rates p={p}")
    rows = studies.vortex_study(2, [20, 40], [p], 0.5, 0.1, emit=say)
    for r in rows:
        rate = r.get("rate")
        if rate is not None:
            assert p - 0.2 <= rate <= p + 1.2, rate
        if not r["dissipation"]:
            assert abs(r["entropy_change"]) < 1e-12


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2), (3, 3)])
def test_diagnostics_kinetic_energy_vs_oracle(dim, p):
    """sbp_diagnostics against the oracle: total entropy, the conserved sums
    and the kinetic energy sum H rho |V|^2 / 2 of the Taylor-Green study."""
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    from tests.gpu_common import state
    say(f"[diagnostics] dim={dim} p={p}")
    desc = wl.vortex2d_mesh(4, warp=0.05) if dim == 2 else wl.tgv_mesh(3)
    m = OracleMesh(desc, p)
    u = state(m, "vortex" if dim == 2 else "tgv", seed=3, jitter=0.01)
    mesh = sbp.Mesh(desc, p)
    d = mesh.diagnostics(torch.from_numpy(u).cuda())
    mesh.check_device()
    mesh.close()
    sch = OracleScheme(m, ph.Gas())
    H = m.H_all()
    ref = np.concatenate([[sch.total_entropy(u)], np.einsum("en,ecn->c", H, u), [sch.kinetic_energy(u)]])
    # the momentum sums of the symmetric fields nearly cancel: their error is
    # taken relative to the sum of magnitudes (V3 = 0 in the Taylor-Green
    # field: that sum and its scale are zero)
    scale = np.concatenate([[abs(ref[0])], np.einsum("en,ecn->c", H, np.abs(u)), [ref[-1]]])
    err = np.abs(d - ref) / np.maximum(scale, np.finfo(float).tiny)
    say("   rel err", err)
    assert d.shape == (m.n_c + 2,) and (err <= 1e-13).all(), err


def test_tgv_history_small():
    """The Taylor-Green history on 3^3 x 6 tetrahedra, p = 2, FP64, Re = 100:
    E_k starts at the oracle's value of the nodal initial field and falls at
    every step (epsilon > 0)."""
    import math
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import studies, workloads as wl
    from tests.gpu_common import state
    say("[tgv history]")
    r = studies.tgv_run(3, 2, steps=6, re=100.0, cfl=0.1, precision="fp64")
    say("   E_k", r["E_k"], "epsilon", r["epsilon"])
    m = OracleMesh(wl.tgv_mesh(3), 2)
    ek0 = OracleScheme(m, ph.Gas()).kinetic_energy(state(m, "tgv")) / (2 * math.pi) ** 3
    assert abs(r["E_k"][0] - ek0) <= 1e-13 * ek0
    assert all(b < a for a, b in zip(r["E_k"], r["E_k"][1:]))
    assert min(r["epsilon"]) > 0 and len(r["t"]) == 7


def test_tgv_dissipation_rate_closed_form():
    """The Navier-Stokes Taylor-Green grid of the benchmark (24^3 x 6
    tetrahedra, p = 3, FP32 residuals, Re = 1600): over the first 20 steps
    the dissipation rate -dE_k/dt stays at its incompressible value at t = 0,
    nu <|omega|^2> = 3 / (4 Re) (the initial vorticity has mean square 3/4),
    within 2% (compressibility at M = 0.1 enters at O(M^2))."""
    import numpy as np
    from paper_2305_07181_amd import studies
    say("[tgv epsilon]")
    r = studies.tgv_run(24, 3, steps=20, re=1600.0, cfl=0.1)
    eps = np.array(r["epsilon"])
    ref = 3.0 / (4.0 * 1600.0)
    say(f"   epsilon mean {eps.mean():.6e} min {eps.min():.6e} max {eps.max():.6e}, 3/(4 Re) {ref:.6e}")
    assert abs(r["E_k"][0] - 0.125) <= 1e-12
    assert np.abs(eps / ref - 1.0).max() <= 0.02
