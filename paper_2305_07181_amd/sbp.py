"""ctypes binding of the C ABI in include/sbp.h (argument marshalling only).

Every step of the residual and the RRK step runs in the HIP library
``libsbp.so``; if it is missing, importing this module raises.

    from paper_2305_07181_amd import sbp
    mesh = sbp.Mesh(desc, degree=2, dissipation=False)   # desc: workloads.* dict
    r = mesh.residual(u)             # u: torch.float64 CUDA tensor [n_elem, n_c, n_p]
    rep = mesh.rrk_step(u, cfl=0.1)  # in place
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsbp.so")

SBP_OK, SBP_EINVAL, SBP_ENOMEM, SBP_EDEVICE, SBP_ENOTSUP, SBP_ENONPHYS, SBP_ERRK = 0, -1, -2, -3, -4, -5, -6
FORM_SPLIT, FORM_HADAMARD = 0, 1
FP64, FP32 = 0, 1
SOURCE_NONE, SOURCE_NS_MMS, SOURCE_VORTEX3D, SOURCE_VORTEX2D = 0, 1, 2, 3
NORM_NODAL, NORM_QUADRATURE = 0, 1

SYMBOLS = ["sbp_setup_mesh", "sbp_mesh_info", "sbp_residual", "sbp_residual_vjp", "sbp_rrk_step",
           "sbp_diagnostics", "sbp_check_device", "sbp_set_time", "sbp_destroy_mesh",
           "sbp_last_error", "sbp_reference_operator", "sbp_use_graphs", "sbp_autotune",
           "sbp_get_launch_shape", "sbp_set_launch_shape", "sbp_set_volume_form", "sbp_set_source",
           "sbp_source_state", "sbp_source_error", "sbp_residual_noalloc", "sbp_time_launches",
           "sbp_launch_times"]


class SbpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sbp error {code}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vert", C.c_int32), ("n_elem", C.c_int32),
                ("vert_xyz", C.POINTER(C.c_double)), ("elem_vert", C.POINTER(C.c_int32)),
                ("p_geom", C.c_int32), ("geom_nodes", C.POINTER(C.c_double)),
                ("period", C.POINTER(C.c_double)), ("elem_degree", C.POINTER(C.c_int32)),
                ("problem_off", C.POINTER(C.c_int32)), ("n_problems", C.c_int32)]


class Physics(C.Structure):
    _fields_ = [("gamma", C.c_double), ("beta", C.c_double), ("form", C.c_int32),
                ("dissipation", C.c_int32), ("viscous", C.c_int32), ("heat_flux", C.c_int32),
                ("mu", C.c_double), ("Pr", C.c_double), ("R", C.c_double), ("precision", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_c", C.c_int32), ("n_elem", C.c_int32),
                ("n_nodes", C.c_int64), ("node_off", C.POINTER(C.c_int64)),
                ("elem_np", C.POINTER(C.c_int32)), ("node_xyz", C.c_void_p),
                ("node_h", C.c_void_p), ("t", C.c_double)]


class RRKReport(C.Structure):
    _fields_ = [("gamma_n", C.c_double), ("dt", C.c_double), ("t", C.c_double),
                ("entropy_before", C.c_double), ("entropy_after", C.c_double),
                ("entropy_rate_e", C.c_double), ("newton_iters", C.c_int32)]


class TuneSlot(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_int32), ("variant", C.c_int32), ("grid", C.c_int32),
                ("n_candidates", C.c_int32), ("ms_builtin", C.c_double), ("ms_best", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("slot", TuneSlot * 8)]


def load_library(path: str = _LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2305_07181_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.sbp_setup_mesh.argtypes = [C.POINTER(MeshDesc), C.POINTER(Physics), P, C.POINTER(P)]
    lib.sbp_mesh_info.argtypes = [P, C.POINTER(Info)]
    lib.sbp_residual.argtypes = [P, P, P, P, P]
    lib.sbp_residual_vjp.argtypes = [P, P, P, P, P]
    lib.sbp_residual_noalloc.argtypes = [P, P, P, P, P]
    lib.sbp_rrk_step.argtypes = [P, P, C.c_double, C.c_double, C.POINTER(RRKReport), P]
    lib.sbp_diagnostics.argtypes = [P, P, C.POINTER(C.c_double), P]
    lib.sbp_check_device.argtypes = [P, P]
    lib.sbp_set_time.argtypes = [P, C.c_double]
    lib.sbp_use_graphs.argtypes = [P, C.c_int]
    lib.sbp_autotune.argtypes = [P, P, P, C.POINTER(TuneReport), P]
    lib.sbp_get_launch_shape.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.sbp_set_launch_shape.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    lib.sbp_set_volume_form.argtypes = [P, P]
    lib.sbp_set_source.argtypes = [P, C.c_int32, P]
    lib.sbp_source_state.argtypes = [P, C.c_double, P, P]
    lib.sbp_source_error.argtypes = [P, P, C.c_double, C.c_int32, P, P]
    lib.sbp_destroy_mesh.argtypes = [P]
    lib.sbp_time_launches.argtypes = [P, C.c_int32]
    lib.sbp_launch_times.argtypes = [P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]
    lib.sbp_last_error.restype = C.c_char_p
    lib.sbp_reference_operator.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    for name in SYMBOLS:
        if name != "sbp_last_error":
            getattr(lib, name).restype = C.c_int
    return lib


# torch is imported before the library is loaded so that one HIP runtime
# serves both: libsbp.so binds to the runtime torch has already loaded.  If
# the library were loaded first, the process would hold two HIP runtimes and
# the library's would find no device.
import torch  # noqa: E402,F401

_lib = load_library()


def _check(rc):
    if rc != SBP_OK:
        raise SbpError(rc, _lib.sbp_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def reference_operator(dim: int, p: int) -> dict:
    """The library's reference operator for (dim, p) (host computation)."""
    n_p = C.c_int32()
    n_f = C.c_int32()
    _check(_lib.sbp_reference_operator(dim, p, C.byref(n_p), C.byref(n_f), None, None, None, None, None, None))
    n_p, n_f = n_p.value, n_f.value
    nodes = np.zeros((n_p, dim))
    h = np.zeros(n_p)
    Q = np.zeros((dim, n_p, n_p))
    E = np.zeros((dim, n_p))
    fn = np.zeros((dim + 1, n_f), dtype=np.int32)
    fw = np.zeros((dim + 1, n_f))
    _check(_lib.sbp_reference_operator(dim, p, None, None, _dp(nodes), _dp(h), _dp(Q), _dp(E), _ip(fn), _dp(fw)))
    return dict(n_p=n_p, n_f=n_f, nodes=nodes, h=h, Q=Q, E=E, facet_nodes=fn, facet_w=fw)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class _DevArray:
    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (int(ptr), False),
                                         "version": 3, "strides": None}


def _device_view(ptr, n):
    import torch
    return torch.as_tensor(_DevArray(ptr, n), device="cuda")


class Mesh:
    """A mesh handle (sbp_setup_mesh) with its physics.

    desc: mesh description dict (workloads.*): dim, vert_xyz, elem_vert,
    period, p_geom, geom_nodes; degree: int or per-element array;
    problem_off: optional element ranges of independent problems."""

    def __init__(self, desc: dict, degree, *, gamma=1.4, beta=2.5, form=FORM_SPLIT, dissipation=False,
                 viscous=False, heat_flux=True, mu=0.0, Pr=0.71, R=1.0, precision=FP64,
                 problem_off=None, stream=None):
        import torch
        self._keep = []
        dim = int(desc["dim"])
        vert = np.ascontiguousarray(desc["vert_xyz"], dtype=np.float64)
        elem = np.ascontiguousarray(desc["elem_vert"], dtype=np.int32)
        period = np.ascontiguousarray(desc["period"], dtype=np.float64)
        ne = len(elem)
        deg = np.ascontiguousarray(np.broadcast_to(np.asarray(degree, dtype=np.int32), (ne,)))
        d = MeshDesc()
        d.dim, d.n_vert, d.n_elem = dim, len(vert), ne
        d.vert_xyz, d.elem_vert, d.period, d.elem_degree = _dp(vert), _ip(elem), _dp(period), _ip(deg)
        self._keep += [vert, elem, period, deg]
        d.p_geom = int(desc.get("p_geom", 1))
        if d.p_geom == 2:
            g = np.ascontiguousarray(desc["geom_nodes"], dtype=np.float64)
            self._keep.append(g)
            d.geom_nodes = _dp(g)
        if problem_off is not None:
            po = np.ascontiguousarray(problem_off, dtype=np.int32)
            self._keep.append(po)
            d.problem_off = _ip(po)
            d.n_problems = len(po) - 1
        else:
            d.n_problems = 1
        ph = Physics(gamma, beta, form, int(dissipation), int(viscous), int(heat_flux), mu, Pr, R, precision)
        self.physics = ph
        self.precision = precision
        self._h = C.c_void_p()
        torch.cuda.init()
        _check(_lib.sbp_setup_mesh(C.byref(d), C.byref(ph), _stream_ptr(stream), C.byref(self._h)))
        info = Info()
        _check(_lib.sbp_mesh_info(self._h, C.byref(info)))
        self.dim, self.n_c, self.n_elem = info.dim, info.n_c, info.n_elem
        self.n_nodes = info.n_nodes
        self.node_off = np.ctypeslib.as_array(info.node_off, shape=(ne + 1,)).copy()
        self.elem_np = np.ctypeslib.as_array(info.elem_np, shape=(ne,)).copy()
        self._node_xyz = info.node_xyz
        self._node_h = info.node_h
        self.uniform = bool((self.elem_np == self.elem_np[0]).all())

    # ------------------------------------------------------------------
    def state_shape(self):
        if not self.uniform:
            return (int(self.n_nodes * self.n_c),)
        return (self.n_elem, self.n_c, int(self.elem_np[0]))

    def node_coords(self):
        """SBP node coordinates computed by the library (a copy), torch
        float64 [n_nodes*dim]; element e at node_off[e]*dim, layout [dim][n_p]."""
        return _device_view(self._node_xyz, int(self.n_nodes * self.dim)).clone()

    def node_weights(self):
        """Diagonal of H_k for all nodes (a copy), torch float64 [n_nodes]."""
        return _device_view(self._node_h, int(self.n_nodes)).clone()

    def residual(self, u, r=None, entropy_rate=False, stream=None):
        import torch
        self._check_state(u)
        rdt = torch.float64 if self.precision == FP64 else torch.float32
        if r is None:
            r = torch.empty(u.shape, dtype=rdt, device=u.device)
        else:
            self._check_state(r, rdt, "r", u.device)
        er = torch.zeros(1, dtype=torch.float64, device=u.device) if entropy_rate else None
        _check(_lib.sbp_residual(self._h, _ptr(u), _ptr(r), _ptr(er) if er is not None else None,
                                 _stream_ptr(stream)))
        return (r, er) if entropy_rate else r

    def residual_noalloc(self, u, r, entropy_rate=None, stream=None):
        """sbp_residual_noalloc: the residual into the caller's r (and the
        entropy rate into the caller's one-element float64 tensor), with the
        library's device scratch in its static array (no allocation)."""
        import torch
        self._check_state(u)
        self._check_state(r, torch.float64 if self.precision == FP64 else torch.float32, "r", u.device)
        if entropy_rate is not None and (entropy_rate.dtype != torch.float64 or not entropy_rate.is_cuda
                                         or entropy_rate.numel() < 1):
            raise ValueError("entropy_rate must be a float64 CUDA tensor of at least one value")
        _check(_lib.sbp_residual_noalloc(self._h, _ptr(u), _ptr(r),
                                         _ptr(entropy_rate) if entropy_rate is not None else None,
                                         _stream_ptr(stream)))
        return r

    def vjp(self, u, lam, ubar=None, stream=None):
        """sbp_residual_vjp: ubar = (dr/du)^T lam, all FP64 (also on FP32
        meshes: the VJP kernels compute in FP64)."""
        import torch
        self._check_state(u)
        self._check_state(lam, torch.float64, "cotangent", u.device)
        if ubar is None:
            ubar = torch.empty_like(u)
        else:
            self._check_state(ubar, torch.float64, "ubar", u.device)
        _check(_lib.sbp_residual_vjp(self._h, _ptr(u), _ptr(lam), _ptr(ubar), _stream_ptr(stream)))
        return ubar

    def rrk_step(self, u, dt=0.0, cfl=0.1, stream=None, report=True):
        """sbp_rrk_step; returns the step report as a dict, or None with
        report=False (then the entropy sums are not computed)."""
        self._check_state(u)
        if not report:
            _check(_lib.sbp_rrk_step(self._h, _ptr(u), float(dt), float(cfl), None, _stream_ptr(stream)))
            return None
        rep = RRKReport()
        _check(_lib.sbp_rrk_step(self._h, _ptr(u), float(dt), float(cfl), C.byref(rep), _stream_ptr(stream)))
        return dict(gamma=rep.gamma_n, dt=rep.dt, t=rep.t, entropy_before=rep.entropy_before,
                    entropy_after=rep.entropy_after, e=rep.entropy_rate_e, iters=rep.newton_iters)

    def autotune(self, u, lam=None, stream=None):
        """sbp_autotune: pick the launch shape of every kernel slot by timing
        (the VJP slots too when a cotangent is given).  Returns one dict per
        slot: kind ("residual"/"vjp"), p (0: batched launch), variant, grid,
        n_candidates, ms_builtin, ms_best."""
        self._check_state(u)
        rep = TuneReport()
        _check(_lib.sbp_autotune(self._h, _ptr(u), _ptr(lam) if lam is not None else None, C.byref(rep),
                                 _stream_ptr(stream)))
        return [dict(kind=("residual", "vjp")[t.kind], p=t.p, variant=t.variant, grid=t.grid,
                     n_candidates=t.n_candidates, ms_builtin=t.ms_builtin, ms_best=t.ms_best)
                for t in rep.slot[:rep.n_slots]]

    def launch_shape(self, kind="residual", p=0):
        """(variant, grid) of one kernel slot (sbp_get_launch_shape)."""
        v, g = C.c_int32(), C.c_int32()
        _check(_lib.sbp_get_launch_shape(self._h, ("residual", "vjp").index(kind), int(p), C.byref(v), C.byref(g)))
        return v.value, g.value

    def set_launch_shape(self, kind="residual", p=0, variant=0, grid=1):
        """Pin the launch shape of one kernel slot (sbp_set_launch_shape)."""
        _check(_lib.sbp_set_launch_shape(self._h, ("residual", "vjp").index(kind), int(p), int(variant), int(grid)))

    def set_volume_form(self, flags=None):
        """Hybrid scheme (sbp_set_volume_form): flags is a uint8 CUDA tensor of
        n_elem values (0 entropy split, 1 Hadamard) that later residuals and
        RRK steps read (its contents may change between calls), or None."""
        import torch
        if flags is not None:
            if flags.dtype != torch.uint8 or not flags.is_cuda or not flags.is_contiguous() \
                    or flags.numel() != self.n_elem:
                raise ValueError("flags must be a contiguous uint8 CUDA tensor of n_elem values")
        _check(_lib.sbp_set_volume_form(self._h, _ptr(flags) if flags is not None else None))
        self._form_flags = flags   # keep the borrowed array alive

    def set_source(self, kind=None, params=None):
        """Fields and source of a study (sbp_set_source): kind SOURCE_NS_MMS
        (default; the manufactured solution, params (rho0, a, c, V0) or None
        for the paper's values), SOURCE_VORTEX3D or SOURCE_VORTEX2D (the
        isentropic vortices of the accuracy studies, no source term; the 2D
        one takes (alpha, xc, yc)) or SOURCE_NONE."""
        kind = SOURCE_NS_MMS if kind is None else int(kind)
        par = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        need = {SOURCE_NS_MMS: 4, SOURCE_VORTEX2D: 3}.get(kind)
        if par is not None and need is not None and par.shape != (need,):
            raise ValueError("params: (rho0, a, c, V0) for the manufactured solution, "
                             "(alpha, xc, yc) for the 2D vortex")
        _check(_lib.sbp_set_source(self._h, kind, _dp(par) if par is not None else None))

    def source_state(self, t, u=None, stream=None):
        """The manufactured fields at the nodes at time t (sbp_source_state)."""
        import torch
        if u is None:
            u = torch.empty(self.state_shape(), dtype=torch.float64, device="cuda")
        self._check_state(u)
        _check(_lib.sbp_source_state(self._h, float(t), _ptr(u), _stream_ptr(stream)))
        return u

    def source_error(self, u, t, norm="quadrature", stream=None):
        """Per component squared L2 error against the manufactured fields at
        time t (sbp_source_error): norm "quadrature" (degree-p fit integrated
        with a degree 3p+1 rule, the paper's studies) or "nodal" (H norm)."""
        self._check_state(u)
        kinds = {"nodal": NORM_NODAL, "quadrature": NORM_QUADRATURE}
        if norm not in kinds:
            raise ValueError("norm must be 'nodal' or 'quadrature'")
        out = np.zeros(self.n_c)
        _check(_lib.sbp_source_error(self._h, _ptr(u), float(t), kinds[norm], _dp(out), _stream_ptr(stream)))
        return out

    def use_graphs(self, enable=True):
        _check(_lib.sbp_use_graphs(self._h, int(bool(enable))))

    def time_launches(self, capacity):
        """sbp_time_launches: the 2D entropy-split kernel records its own
        start and end for the next `capacity` sbp_residual calls (0: stop)."""
        _check(_lib.sbp_time_launches(self._h, int(capacity)))

    def launch_times(self, max_n=65536):
        """sbp_launch_times: the recorded kernel durations in ms (waits for
        them), oldest first; clears the record."""
        out = np.zeros(max(1, int(max_n)))
        n = C.c_int32()
        _check(_lib.sbp_launch_times(self._h, _dp(out), int(max_n), C.byref(n)))
        return out[:n.value].copy()

    def diagnostics(self, u, stream=None):
        """sbp_diagnostics: [sum H s, sum H u per component (n_c values),
        sum H rho |V|^2 / 2]."""
        self._check_state(u)
        out = np.zeros(self.n_c + 2)
        _check(_lib.sbp_diagnostics(self._h, _ptr(u), _dp(out), _stream_ptr(stream)))
        return out

    def check_device(self, stream=None):
        _check(_lib.sbp_check_device(self._h, _stream_ptr(stream)))

    def set_time(self, t):
        _check(_lib.sbp_set_time(self._h, float(t)))

    def _check_state(self, u, dtype=None, what="state", device=None):
        """Raise ValueError unless u is a contiguous CUDA tensor of the state
        size with the given dtype (float64 by default) on `device`."""
        import torch
        dtype = torch.float64 if dtype is None else dtype
        if not isinstance(u, torch.Tensor) or u.dtype != dtype or not u.is_cuda or not u.is_contiguous():
            raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor")
        if device is not None and u.device != device:
            raise ValueError(f"{what} is on {u.device}, the state on {device}")
        if u.numel() != self.n_nodes * self.n_c:
            raise ValueError(f"{what} has {u.numel()} values, expected {self.n_nodes * self.n_c}")

    def close(self):
        if self._h:
            _lib.sbp_destroy_mesh(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Residual(torch.autograd.Function):
    """r = du/dt of a mesh handle as a differentiable torch operation:
    forward calls sbp_residual, backward calls sbp_residual_vjp (the
    hand-written vector-Jacobian kernels).  Only argument marshalling happens
    here; the cotangent is passed to the library as FP64 (the VJP kernels
    compute in FP64 also for FP32 meshes).  Use through :func:`residual`."""

    @staticmethod
    def forward(ctx, u, mesh):
        ud = u.detach()
        ctx.mesh = mesh
        ctx.save_for_backward(ud)
        return mesh.residual(ud)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_r):
        (u,) = ctx.saved_tensors
        lam = grad_r
        if lam.dtype != torch.float64 or not lam.is_contiguous():
            lam = lam.to(torch.float64).contiguous()
        return ctx.mesh.vjp(u, lam), None


def residual(mesh: "Mesh", u):
    """Differentiable residual r(u) of `mesh` (see :class:`Residual`)."""
    return Residual.apply(u, mesh)
