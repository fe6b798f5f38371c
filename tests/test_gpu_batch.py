"""Batched 2D problems (mixed degree, one persistent launch per call): the
residual and its VJP against the oracle run problem by problem, and a
finite-difference check of the VJP on the whole batch."""
import numpy as np
import pytest

from tests.gpu_common import rel_err_per_component, say, state

pytestmark = pytest.mark.gpu

SMALL = [dict(p=1, nx=2, ny=3), dict(p=2, nx=3, ny=3), dict(p=3, nx=2, ny=2),
         dict(p=4, nx=3, ny=2), dict(p=2, nx=4, ny=4), dict(p=4, nx=2, ny=3)]


def _batch(specs, warp):
    from oracle.geometry import OracleMesh
    from paper_2305_07181_amd import workloads as wl
    desc, deg, off = wl.batch_mesh(specs, warp=warp)
    meshes, states = [], []
    for b, sp in enumerate(specs):
        m = OracleMesh(wl.sub_mesh(desc, off[b], off[b + 1]), sp["p"])
        meshes.append(m)
        states.append(state(m, "batch", seed=1000 + b))
    return desc, deg, off, meshes, states


def _flat(mesh, off, parts):
    """Per-problem arrays [ne_b, n_c, n_p_b] -> the library's flat layout."""
    out = np.zeros(int(mesh.n_nodes * mesh.n_c))
    for b, a in enumerate(parts):
        for k in range(a.shape[0]):
            e = off[b] + k
            o = int(mesh.node_off[e] * mesh.n_c)
            out[o:o + a[k].size] = a[k].ravel()
    return out


def _split(mesh, off, flat, shapes):
    parts = []
    for b, shp in enumerate(shapes):
        a = np.zeros(shp)
        for k in range(shp[0]):
            o = int(mesh.node_off[off[b] + k] * mesh.n_c)
            a[k] = flat[o:o + a[k].size].reshape(shp[1:])
        parts.append(a)
    return parts


@pytest.mark.parametrize("diss", [False, True])
def test_batched_residual_vs_oracle(diss):
    import torch
    from oracle import physics as ph
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say(f"[batch residual] diss={diss}")
    desc, deg, off, meshes, states = _batch(SMALL, 0.05)
    mesh = sbp.Mesh(desc, deg, dissipation=diss, problem_off=off)
    u = torch.from_numpy(_flat(mesh, off, states)).cuda()
    r, er = mesh.residual(u, entropy_rate=True)
    mesh.check_device()
    parts = _split(mesh, off, r.cpu().numpy(), [s.shape for s in states])
    total = 0.0
    scale = 0.0
    for b, (m, ub) in enumerate(zip(meshes, states)):
        sch = OracleScheme(m, ph.Gas(), dissipation=diss)
        ro = sch(ub)
        err = rel_err_per_component(parts[b], ro)
        say(f"   problem {b} p={SMALL[b]['p']} ne={m.ne}: rel err {err.max():.2e}")
        assert (err <= 1e-12).all(), (b, err)
        total += sch.entropy_rate(ub, ro)
        scale += np.sum(np.abs(ro))
    assert abs(float(er.cpu()[0]) - total) <= 1e-12 * scale
    mesh.close()


def test_batched_vjp_vs_oracle():
    import torch
    from oracle import physics as ph
    from oracle.jacobian import vjp_elements
    from oracle.residual import OracleScheme
    from paper_2305_07181_amd import sbp
    say("[batch vjp]")
    desc, deg, off, meshes, states = _batch(SMALL, 0.05)
    lams = [np.random.default_rng(2000 + b).standard_normal(s.shape) for b, s in enumerate(states)]
    mesh = sbp.Mesh(desc, deg, dissipation=True, problem_off=off)
    u = torch.from_numpy(_flat(mesh, off, states)).cuda()
    lam = torch.from_numpy(_flat(mesh, off, lams)).cuda()
    ub = mesh.vjp(u, lam)
    mesh.check_device()
    parts = _split(mesh, off, ub.cpu().numpy(), [s.shape for s in states])
    for b, m in enumerate(meshes):
        sch = OracleScheme(m, ph.Gas(), dissipation=True)
        els = sorted({0, m.ne // 2, m.ne - 1})
        ref = vjp_elements(sch, states[b], lams[b], els)
        sc = max(np.abs(ref[e]).max() for e in els)
        err = max(np.abs(parts[b][e] - ref[e]).max() for e in els) / sc
        say(f"   problem {b}: rel err {err:.2e}")
        assert err <= 1e-12, (b, err)
    mesh.close()


def test_batched_fd_check():
    """Forward + VJP of 16 problems drawn like the 48-problem batch (smaller
    grids), lambda ~ N(0,1) (seed 2000+b), FD along a random direction
    (seed 3000+b), h = 1e-6 (FP64)."""
    import torch
    from paper_2305_07181_amd import sbp, workloads as wl
    say("[batch fd]")
    specs = [dict(sp, nx=max(2, sp["nx"] // 4), ny=max(2, sp["ny"] // 4)) for sp in wl.batch_problem_specs(16, 0)]
    desc, deg, off, meshes, states = _batch(specs, 0.0)
    lams = [np.random.default_rng(2000 + b).standard_normal(s.shape) for b, s in enumerate(states)]
    dirs = [np.random.default_rng(3000 + b).standard_normal(s.shape) * np.abs(s) for b, s in enumerate(states)]
    mesh = sbp.Mesh(desc, deg, problem_off=off)
    u, lam, v = (torch.from_numpy(_flat(mesh, off, a)).cuda() for a in (states, lams, dirs))
    ub = mesh.vjp(u, lam)
    h = 1e-6
    fd = float(torch.sum(lam * (mesh.residual(u + h * v) - mesh.residual(u - h * v))) / (2 * h))
    ad = float(torch.sum(v * ub))
    say("   fd", fd, "ad", ad, "rel", abs(fd - ad) / abs(ad))
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    mesh.close()
