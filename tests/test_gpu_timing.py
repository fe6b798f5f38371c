"""Launch timing (sbp_time_launches / sbp_launch_times): the recorded
durations of the residual kernels, in call order, without changing the
residual; records stop at the capacity and are cleared when read; the other
entry points are not timed."""
import numpy as np
import pytest

from tests.gpu_common import say, state

pytestmark = pytest.mark.gpu


def test_launch_times_record_the_residual_kernels():
    import torch
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[timing] 2D p=3 and 3D p=2")
    for desc, p in ((wl.vortex2d_mesh(16, warp=0.05), 3), (wl.periodic_tet_mesh(4, 1.0), 2)):
        m = OracleMesh(desc, p)
        u = torch.from_numpy(state(m, "random", seed=5, jitter=0.01)).cuda()
        mesh = sbp.Mesh(desc, p, dissipation=True)
        r0 = mesh.residual(u)
        mesh.time_launches(3)
        rs = [mesh.residual(u) for _ in range(5)]
        ms = mesh.launch_times()
        say(f"   dim {mesh.dim}: {np.array2string(ms, precision=4)} ms")
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
