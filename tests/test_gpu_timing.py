"""Launch timing (sbp_time_launches / sbp_launch_times): the durations the
2D entropy-split kernel records itself, in call order, without changing the
residual; records stop at the capacity and are cleared when read; the other
entry points are not timed; other meshes are refused."""
import numpy as np
import pytest

from tests.gpu_common import say, state

pytestmark = pytest.mark.gpu


def test_launch_times_record_the_residual_kernels():
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[timing] 2D p=3, FP64 and FP32")
    for desc, p, prec in ((wl.vortex2d_mesh(16, warp=0.05), 3, 0), (wl.vortex2d_mesh(8), 1, 1)):
        m = OracleMesh(desc, p)
        u = torch.from_numpy(state(m, "random", seed=5, jitter=0.01)).cuda()
        mesh = sbp.Mesh(desc, p, dissipation=True, precision=prec)
        r0 = mesh.residual(u)
        mesh.time_launches(3)
        rs = [mesh.residual(u) for _ in range(5)]
        ms = mesh.launch_times()
        say(f"   p {p} precision {prec}: {np.array2string(ms, precision=4)} ms")
        assert len(ms) == 3 and (ms > 0).all() and (ms < 1000).all()
        assert all(torch.equal(r, r0) for r in rs)
        mesh.residual(u)
        assert len(mesh.launch_times()) == 1          # recording continues after a read
        mesh.rrk_step(u.clone(), cfl=0.1)              # not timed
        mesh.vjp(u, u)
        assert len(mesh.launch_times()) == 0
        mesh.time_launches(0)
        mesh.residual(u)
        assert len(mesh.launch_times()) == 0
        with pytest.raises(sbp.SbpError):
            mesh.time_launches(-1)
        mesh.check_device()
        mesh.close()


def test_launch_timing_batched_launch():
    """A mesh of several degrees: one record per call (its one batched launch)."""
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[timing] batched launch")
    desc = wl.vortex2d_mesh(8, warp=0.05)
    d4, deg, off = wl.copies_mesh(desc, (1, 3))
    parts = [state(OracleMesh(desc, p), "random", seed=6 + p, jitter=0.01) for p in (1, 3)]
    u = torch.from_numpy(np.concatenate([q.ravel() for q in parts])).cuda()
    mesh = sbp.Mesh(d4, deg, problem_off=off)
    r0 = mesh.residual(u)
    mesh.time_launches(8)
    rs = [mesh.residual(u) for _ in range(3)]
    ms = mesh.launch_times()
    assert len(ms) == 3 and (ms > 0).all()
    assert all(torch.equal(r, r0) for r in rs)
    mesh.check_device()
    mesh.close()


def test_launch_timing_refused_where_not_recorded():
    """Tetrahedra and the Hadamard form run other kernels: SBP_ENOTSUP."""
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[timing] refusals")
    cases = [(wl.periodic_tet_mesh(2, 1.0), 2, {}), (wl.vortex2d_mesh(4), 2, dict(form=sbp.FORM_HADAMARD))]
    for desc, p, kw in cases:
        mesh = sbp.Mesh(desc, p, **kw)
        with pytest.raises(sbp.SbpError) as ei:
            mesh.time_launches(4)
        assert ei.value.code == sbp.SBP_ENOTSUP
        mesh.time_launches(0)
        mesh.close()
