"""sbp_residual_noalloc (the residual for callers that cannot allocate: its
scratch lives in the library's static device array) against sbp_residual:
two calls in a row, the second on a smaller mesh, bitwise equal residuals
and entropy rates; the hybrid flags, the manufactured source (whose
entropy rate uses the node partials in the same array) and a mesh of four
degree classes (one batched launch, its per-workgroup partials in the same
array) included."""
import numpy as np
import pytest

from tests.gpu_common import say, state

pytestmark = pytest.mark.gpu


def _pair(mesh, u, **kw):
    import torch
    r_ref, e_ref = mesh.residual(u, entropy_rate=True)
    r = torch.full_like(r_ref, float("nan"))
    e = torch.full((1,), float("nan"), dtype=torch.float64, device=u.device)
    mesh.residual_noalloc(u, r, e)
    torch.cuda.synchronize()
    return r_ref, e_ref, r, e


def _batch_state(mesh, off):
    """Vortex state on each copy of a mesh of grid copies (workloads.copies_mesh)."""
    from paper_2305_07181_amd import workloads as wl
    x = mesh.node_coords().cpu().numpy()
    u = np.zeros(int(mesh.n_nodes * mesh.n_c))
    for b in range(len(off) - 1):
        n_p = int(mesh.elem_np[off[b]])
        e0, e1 = int(off[b]), int(off[b + 1])
        lo, hi = int(mesh.node_off[e0]), int(mesh.node_off[e1])
        X = np.moveaxis(x[lo * 2:hi * 2].reshape(e1 - e0, 2, n_p), 1, 0)
        rho, V, pr = wl.isentropic_vortex(X)
        u[lo * 4:hi * 4] = np.moveaxis(wl.conservative(rho, V, pr), 0, 1).ravel()
    return u


def test_noalloc_batched_launch_two_calls():
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    for n in (8, 4):                    # second call: a smaller input
        say(f"[noalloc] tri-batch p=1..4 n={n}")
        desc, deg, off = wl.copies_mesh(wl.vortex2d_mesh(n, warp=0.05), (1, 2, 3, 4))
        mesh = sbp.Mesh(desc, deg, problem_off=off)
        u = _batch_state(mesh, off)
        ud = torch.from_numpy(u * (1 + 0.01 * np.random.default_rng(n).standard_normal(u.shape))).cuda()
        r_ref, e_ref, r, e = _pair(mesh, ud)
        mesh.check_device()
        assert torch.equal(r, r_ref), float((r - r_ref).abs().max())
        assert torch.equal(e, e_ref), (float(e), float(e_ref))
        say("   bitwise equal; entropy rate", float(e))
        mesh.close()


@pytest.mark.parametrize("case", ["tri-split", "tet-hybrid", "tet-ns-source"])
def test_noalloc_matches_residual_two_calls(case):
    import torch
    from oracle import physics as ph
    from oracle.geometry import OracleMesh
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp, workloads as wl
    for n_big, n_small in [(12, 4)] if case == "tri-split" else [(3, 2)]:
        for n in (n_big, n_small):      # second call: a smaller input
            say(f"[noalloc] {case} n={n}")
            if case == "tri-split":
                desc, p, kw = wl.vortex2d_mesh(n, warp=0.05), 3, dict(dissipation=True)
            elif case == "tet-hybrid":
                desc, p, kw = wl.periodic_tet_mesh(n, 1.0), 2, dict(dissipation=True)
            else:
                desc, p, kw = wl.mms_mesh3d(n), 2, dict(viscous=True, mu=0.01)
            m = OracleMesh(desc, p)
            mesh = sbp.Mesh(desc, p, **kw)
            if case == "tet-ns-source":
                mesh.set_source(sbp.SOURCE_NS_MMS)
                ud = mesh.source_state(0.0)
                ud.mul_(torch.from_numpy(1 + 0.01 * np.random.default_rng(n).standard_normal(tuple(ud.shape))).cuda())
                u = ud.cpu().numpy()
            else:
                u = state(m, "random", seed=50 + n, jitter=0.01)
                ud = torch.from_numpy(u).cuda()
            if case == "tet-hybrid":
                flags = torch.from_numpy(np.random.default_rng(n).integers(0, 2, m.ne).astype(np.uint8)).cuda()
                mesh.set_volume_form(flags)
            r_ref, e_ref, r, e = _pair(mesh, ud)
            mesh.check_device()
            assert torch.equal(r, r_ref), float((r - r_ref).abs().max())
            assert torch.equal(e, e_ref), (float(e), float(e_ref))
            if case == "tri-split":
                # and the oracle's residual at the parity bar
                sch = OracleScheme(m, ph.Gas(), dissipation=True)
                ro = sch(u)
                err = np.abs(r.cpu().numpy() - ro).max(axis=(0, 2)) / np.abs(ro).max(axis=(0, 2))
                assert (err <= 1e-12).all(), err
            say("   bitwise equal; entropy rate", float(e))
            mesh.close()
