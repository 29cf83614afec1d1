"""Python binding of libdgthermo (the C ABI declared in include/dgthermo.h).

Argument marshalling only: every step of R(u), J(u)v and the implicit step runs in
the library's HIP kernels. PyTorch provides device memory and the current stream.
The library is loaded from this package directory; importing fails loudly if it
has not been built (python __graft_entry__.py).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdgthermo.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError("libdgthermo.so is not built: run `python __graft_entry__.py` (hipcc, gfx950)")
_lib = C.CDLL(_LIB_PATH)

DG_OK, DG_ERR_ARG, DG_ERR_ALLOC, DG_ERR_HIP, DG_ERR_NOCONV, DG_ERR_NAN, DG_ERR_UNSUPPORTED = range(7)
DG_F64, DG_F32, DG_BF16, DG_F64_FD = 0, 1, 2, 3
_PREC = {"f64": DG_F64, "f32": DG_F32, "bf16": DG_BF16, "f64_fd": DG_F64_FD}


class DgError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.dg_last_error().decode(errors="replace")
        super().__init__("%s failed (status %d): %s" % (where, code, msg))
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_int32), ("n_ang", C.c_int32), ("n_rad", C.c_int32),
                ("r_bot", C.c_double), ("r_top", C.c_double), ("stretch", C.c_double),
                ("n_col", C.c_int32), ("col_nelem", C.POINTER(C.c_int32)), ("col_p", C.POINTER(C.c_int32)),
                ("col_stretch", C.POINTER(C.c_double))]


class Physics(C.Structure):
    _fields_ = [("gamma", C.c_double), ("Gr", C.c_double), ("Pr", C.c_double), ("Fr", C.c_double),
                ("m", C.c_double), ("nu_r", C.c_double), ("alpha_r", C.c_double), ("alpha0c", C.c_double),
                ("lam", C.c_double), ("T_bot", C.c_double), ("r_ref", C.c_double), ("omega", C.c_double * 3),
                ("heat_amp", C.c_double), ("heat_qm", C.c_double), ("heat_rm", C.c_double), ("heat_H", C.c_double),
                ("sun_lat", C.c_double), ("sun_lon0", C.c_double), ("sun_rate", C.c_double),
                ("bc_mode", C.c_int32), ("bc_state", C.c_double * 5),
                ("col_heat_amp", C.POINTER(C.c_double)), ("col_heat_qm", C.POINTER(C.c_double)),
                ("col_heat_rm", C.POINTER(C.c_double)), ("col_heat_H", C.POINTER(C.c_double)),
                ("col_lam", C.POINTER(C.c_double)),
                ("heating_model", C.c_int32), ("euv_eps", C.c_double), ("euv_f107", C.c_double),
                ("euv_sun_dist", C.c_double), ("euv_day", C.c_double), ("euv_chi", C.c_double * 4),
                ("euv_q_scale", C.c_double), ("euv_col_scale", C.c_double),
                ("col_alpha0c", C.POINTER(C.c_double)), ("col_site", C.POINTER(C.c_double)),
                ("col_euv_eps", C.POINTER(C.c_double)), ("col_euv_f107", C.POINTER(C.c_double)),
                ("composition", C.c_int32), ("comp_a", C.c_double * 6), ("comp_b", C.c_double * 6)]


class SolverOpts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("gmres_m", C.c_int32), ("max_newton", C.c_int32),
                ("max_restarts", C.c_int32), ("newton_rtol", C.c_double), ("gmres_rtol", C.c_double),
                ("jvp_prec", C.c_int32), ("precond", C.c_int32), ("guess", C.c_int32), ("forcing", C.c_int32),
                ("filter_rate", C.c_double), ("n_rb", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("newton_its", C.c_int32 * 3), ("gmres_its", C.c_int32 * 3), ("fallback", C.c_int32 * 3),
                ("res0", C.c_double * 3), ("res", C.c_double * 3), ("ref", C.c_double * 3),
                ("guess_scale", C.c_double * 3), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k != "seconds" else self.seconds) for k, _ in self._fields_}


_vp = C.c_void_p
_lib.dg_last_error.restype = C.c_char_p
_lib.dg_version.restype = C.c_int32
_lib.dg_mesh_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(Physics), _vp, C.POINTER(_vp)]
_lib.dg_mesh_destroy.argtypes = [_vp]
_lib.dg_mesh_set_physics.argtypes = [_vp, C.POINTER(Physics)]
_lib.dg_mesh_info.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)]
_lib.dg_mesh_nodes.argtypes = [_vp, C.POINTER(C.c_double), C.c_int64]
_lib.dg_mesh_col_offsets.argtypes = [_vp, C.POINTER(C.c_int64), C.c_int64]
_lib.dg_residual.argtypes = [_vp, C.c_double, _vp, _vp, C.c_int64, _vp]
_lib.dg_residual_noalloc.argtypes = [_vp, C.c_double, _vp, _vp, C.c_int64, _vp]
_lib.dg_jvp.argtypes = [_vp, C.c_double, _vp, _vp, _vp, C.c_int64, C.c_int32, _vp]
_lib.dg_implicit_step.argtypes = [_vp, C.c_double, C.c_double, _vp, C.c_int64, C.POINTER(SolverOpts),
                                  C.POINTER(StepStats), _vp]
_lib.dg_columns_integrate.argtypes = [_vp, C.c_double, C.c_double, C.c_int32, _vp, C.c_int64,
                                      C.POINTER(SolverOpts), C.POINTER(C.c_int32), C.POINTER(C.c_int32), _vp]
_fp = C.POINTER(C.c_float)
_lib.dg_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, _fp, C.POINTER(_vp)]
_lib.dg_mlp_destroy.argtypes = [_vp]
_lib.dg_mlp_param_count.argtypes = [_vp]
_lib.dg_mlp_param_count.restype = C.c_int64
_lib.dg_mlp_get_params.argtypes = [_vp, _fp, C.c_int64]
_lib.dg_mlp_forward.argtypes = [_vp, _vp, C.c_int64, _vp, _vp]
_lib.dg_mlp_grad.argtypes = [_vp, _vp, _vp, C.c_int64, C.POINTER(C.c_double), _fp, _vp]
_lib.dg_mlp_adam_step.argtypes = [_vp, C.c_float, C.c_float, C.c_float, C.c_float, _vp]
_lib.dg_affine_rows.argtypes = [_vp, C.c_int64, C.c_int32, _vp, _vp, _vp]
_lib.dg_warmstart_set.argtypes = [_vp, _vp, _fp, _fp, _fp, _fp]
_lib.dg_warmstart_record.argtypes = [_vp, _vp, _vp, C.c_int64, C.c_int32]
_lib.dg_warmstart_recorded.argtypes = [_vp, C.POINTER(C.c_int64)]
_lib.dg_profile_enable.argtypes = [_vp, C.c_int32]
_lib.dg_set_option.argtypes = [_vp, C.c_char_p, C.c_int64]
_lib.dg_profile_read.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32, C.c_int32]
for _f in ("dg_mesh_create", "dg_mesh_destroy", "dg_mesh_set_physics", "dg_mesh_info", "dg_mesh_nodes",
           "dg_mesh_col_offsets", "dg_residual", "dg_residual_noalloc", "dg_jvp", "dg_implicit_step",
           "dg_profile_enable",
           "dg_profile_read", "dg_set_option", "dg_columns_integrate", "dg_mlp_create", "dg_mlp_destroy",
           "dg_mlp_get_params", "dg_mlp_forward", "dg_mlp_grad", "dg_mlp_adam_step", "dg_affine_rows",
           "dg_warmstart_set", "dg_warmstart_record", "dg_warmstart_recorded"):
    getattr(_lib, _f).restype = C.c_int32

EXPORTED = ["dg_mesh_create", "dg_mesh_destroy", "dg_mesh_set_physics", "dg_mesh_info", "dg_mesh_nodes",
            "dg_mesh_col_offsets", "dg_residual", "dg_jvp", "dg_implicit_step", "dg_last_error", "dg_version",
            "dg_profile_enable", "dg_profile_read", "dg_set_option", "dg_columns_integrate", "dg_mlp_create",
            "dg_mlp_destroy", "dg_mlp_param_count", "dg_mlp_get_params", "dg_mlp_forward", "dg_mlp_grad",
            "dg_mlp_adam_step", "dg_affine_rows", "dg_warmstart_set", "dg_warmstart_record", "dg_warmstart_recorded",
            "dg_residual_noalloc"]
PROFILE_SLOTS = {0: "shell_pass1_R", 1: "shell_pass2_R", 2: "shell_pass1_jvp64", 3: "shell_pass2_jvp64",
                 4: "shell_pass1_jvp32", 5: "shell_pass2_jvp32", 6: "columns_R", 7: "columns_jvp64",
                 8: "columns_jvp32", 9: "gmres_arnoldi", 10: "bjac_build", 11: "bjac_apply", 12: "vector_ops",
                 13: "columns_batch", 14: "shell_pass1_jvpbf16", 15: "shell_pass2_jvpbf16"}


def _check(code, where):
    if code != DG_OK:
        raise DgError(code, where)


def _dbl_array(x):
    if x is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def make_physics(phys: dict, col_phys: dict | None = None):
    """fill the C struct from a plain parameter dict; returns (struct, keep-alive list)"""
    P = Physics()
    for k in ("gamma", "Gr", "Pr", "Fr", "m", "nu_r", "alpha_r", "alpha0c", "lam", "T_bot", "r_ref",
              "heat_amp", "heat_qm", "heat_rm", "heat_H", "sun_lat", "sun_lon0", "sun_rate"):
        setattr(P, k, float(phys[k]))
    P.omega = (C.c_double * 3)(*[float(x) for x in phys["omega"]])
    P.bc_mode = int(phys.get("bc_mode", 0))
    bs = list(phys.get("bc_state", [0.0] * 5)) + [0.0] * 5
    P.bc_state = (C.c_double * 5)(*[float(x) for x in bs[:5]])
    P.heating_model = int(phys.get("heating_model", 0))
    if P.heating_model == 1:
        for k in ("euv_eps", "euv_f107", "euv_sun_dist", "euv_day", "euv_q_scale", "euv_col_scale"):
            setattr(P, k, float(phys[k]))
        P.euv_chi = (C.c_double * 4)(*[float(x) for x in phys.get("euv_chi", [0.0] * 4)])
    P.composition = int(phys.get("composition", 0))
    if P.composition:
        P.comp_a = (C.c_double * 6)(*[float(x) for x in phys["comp_a"]])
        P.comp_b = (C.c_double * 6)(*[float(x) for x in phys["comp_b"]])
    keep = []
    if col_phys:
        for key, field in (("heat_amp", "col_heat_amp"), ("heat_qm", "col_heat_qm"), ("heat_rm", "col_heat_rm"),
                           ("heat_H", "col_heat_H"), ("lam", "col_lam"), ("alpha0c", "col_alpha0c"),
                           ("site", "col_site"), ("euv_eps", "col_euv_eps"), ("euv_f107", "col_euv_f107")):
            if key in col_phys:
                arr, ptr = _dbl_array(col_phys[key])
                keep.append(arr)
                setattr(P, field, ptr)
    return P, keep


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _ptr(t, dtype=None):
    import torch
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return C.c_void_p(t.data_ptr())


class Mesh:
    """A cubed-sphere shell or a batch of 1D radial columns held by the library."""

    def __init__(self, desc: MeshDesc, phys: dict, col_phys=None, stream=None, _keep=()):
        self._h = C.c_void_p()
        P, keep = make_physics(phys, col_phys)
        self.phys = dict(phys)
        _check(_lib.dg_mesh_create(C.byref(desc), C.byref(P), _stream(stream), C.byref(self._h)), "dg_mesh_create")
        n_dof, n_elem, nf, dim = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        _check(_lib.dg_mesh_info(self._h, C.byref(n_dof), C.byref(n_elem), C.byref(nf), C.byref(dim)), "dg_mesh_info")
        self.n_dof, self.n_elem, self.n_fields, self.dim = n_dof.value, n_elem.value, nf.value, dim.value
        self.kind = desc.kind
        self.p = desc.p
        self.n_col = desc.n_col

    @classmethod
    def shell(cls, p, n_ang, n_rad, r_bot, r_top, stretch, phys, stream=None):
        d = MeshDesc(kind=1, p=p, n_ang=n_ang, n_rad=n_rad, r_bot=r_bot, r_top=r_top, stretch=stretch, n_col=0)
        return cls(d, phys, None, stream)

    @classmethod
    def columns(cls, nelem, p, r_bot, r_top, stretch, phys, col_phys=None, stream=None):
        """stretch: one growth ratio for every column, or an array with one per column"""
        ne = np.ascontiguousarray(np.asarray(nelem, dtype=np.int32))
        pp = np.ascontiguousarray(np.broadcast_to(np.asarray(p, dtype=np.int32), ne.shape))
        sa = np.ascontiguousarray(np.broadcast_to(np.asarray(stretch, dtype=np.float64), ne.shape))
        d = MeshDesc(kind=0, p=0, n_ang=0, n_rad=0, r_bot=r_bot, r_top=r_top, stretch=float(sa[0]), n_col=len(ne),
                     col_nelem=ne.ctypes.data_as(C.POINTER(C.c_int32)),
                     col_p=pp.ctypes.data_as(C.POINTER(C.c_int32)),
                     col_stretch=sa.ctypes.data_as(C.POINTER(C.c_double)))
        m = cls(d, phys, col_phys, stream)
        m.col_nelem, m.col_p, m.col_stretch = ne, pp, sa
        return m

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.dg_mesh_destroy(h)
            self._h = C.c_void_p()

    def set_physics(self, phys, col_phys=None):
        P, keep = make_physics(phys, col_phys)
        _check(_lib.dg_mesh_set_physics(self._h, C.byref(P)), "dg_mesh_set_physics")
        self.phys = dict(phys)

    def set_option(self, name, value):
        _check(_lib.dg_set_option(self._h, name.encode(), int(value)), "dg_set_option")

    def profile(self, on=True):
        _check(_lib.dg_profile_enable(self._h, 1 if on else 0), "dg_profile_enable")

    def profile_read(self, reset=True):
        """{slot name: (total ms, launches)} of the launches timed since the last reset"""
        ms = (C.c_double * 16)()
        cnt = (C.c_int64 * 16)()
        _check(_lib.dg_profile_read(self._h, ms, cnt, 16, 1 if reset else 0), "dg_profile_read")
        return {PROFILE_SLOTS.get(i, str(i)): (ms[i], cnt[i]) for i in range(16) if cnt[i]}

    def nodes(self):
        nn = self.n_dof // self.n_fields
        out = np.zeros(nn * self.dim)
        _check(_lib.dg_mesh_nodes(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), out.size), "dg_mesh_nodes")
        return out.reshape(-1, self.dim) if self.dim == 3 else out

    def col_offsets(self):
        out = np.zeros(self.n_col + 1, dtype=np.int64)
        _check(_lib.dg_mesh_col_offsets(self._h, out.ctypes.data_as(C.POINTER(C.c_int64)), out.size),
               "dg_mesh_col_offsets")
        return out

    def residual(self, u, t=0.0, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(u)
        if out.numel() != u.numel():
            raise ValueError("out must have as many elements as u")
        _check(_lib.dg_residual(self._h, float(t), _ptr(u, torch.float64), _ptr(out, torch.float64), u.numel(),
                                _stream(stream)), "dg_residual")
        return out

    def residual_noalloc(self, u, out, t=0.0, stream=None):
        """R(u) into the caller's `out` through dg_residual_noalloc (the library allocates
        nothing; the face traces use its per-GPU scratch array)"""
        import torch
        if out.numel() != u.numel():
            raise ValueError("out must have as many elements as u")
        _check(_lib.dg_residual_noalloc(self._h, float(t), _ptr(u, torch.float64), _ptr(out, torch.float64),
                                        u.numel(), _stream(stream)), "dg_residual_noalloc")
        return out

    def jvp(self, u, v, t=0.0, prec="f64", out=None, stream=None):
        import torch
        dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32, "f64_fd": torch.float64}[prec]
        if out is None:
            out = torch.empty(self.n_dof, dtype=dt, device=u.device)
        if not (u.numel() == v.numel() == out.numel()):
            raise ValueError("u, v and out must have the same number of elements")
        _check(_lib.dg_jvp(self._h, float(t), _ptr(u, torch.float64), _ptr(v, dt), _ptr(out, dt), u.numel(),
                           _PREC[prec], _stream(stream)), "dg_jvp")
        return out

    def implicit_step(self, u, t, dt, scheme=33, gmres_m=30, max_newton=20, max_restarts=20, newton_rtol=1e-8,
                      gmres_rtol=1e-3, jvp_prec="f64", precond=1, guess=0, filter_rate=0.0, forcing=0, n_rb=0,
                      stream=None):
        import torch
        o = SolverOpts(scheme=scheme, gmres_m=gmres_m, max_newton=max_newton, max_restarts=max_restarts,
                       newton_rtol=newton_rtol, gmres_rtol=gmres_rtol, jvp_prec=_PREC[jvp_prec], precond=precond,
                       guess=guess, forcing=forcing, filter_rate=filter_rate, n_rb=n_rb)
        st = StepStats()
        code = _lib.dg_implicit_step(self._h, float(t), float(dt), _ptr(u, torch.float64), u.numel(), C.byref(o),
                                     C.byref(st), _stream(stream))
        _check(code, "dg_implicit_step")
        return st.as_dict()


def _columns_integrate(self, u, t0, dt, n_steps, scheme=33, max_newton=20, newton_rtol=1e-8, filter_rate=0.0,
                       stream=None, raise_on_failure=True):
    """advance every column by n_steps DIRK steps in one persistent launch; returns
    (Newton iterations per column, status per column)"""
    import torch
    o = SolverOpts(scheme=scheme, gmres_m=1, max_newton=max_newton, max_restarts=1, newton_rtol=newton_rtol,
                   gmres_rtol=1e-3, jvp_prec=DG_F64, precond=0, guess=0, filter_rate=filter_rate)
    its = np.zeros(self.n_col, dtype=np.int32)
    st = np.zeros(self.n_col, dtype=np.int32)
    code = _lib.dg_columns_integrate(self._h, float(t0), float(dt), int(n_steps), _ptr(u, torch.float64), u.numel(),
                                     C.byref(o), its.ctypes.data_as(C.POINTER(C.c_int32)),
                                     st.ctypes.data_as(C.POINTER(C.c_int32)), _stream(stream))
    if code != DG_OK and raise_on_failure:
        raise DgError(code, "dg_columns_integrate")
    return its, st


Mesh.columns_integrate = _columns_integrate


def _f32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Network:
    """the warm-start network n_in -> 128 -> 128 -> n_out held by the library"""

    def __init__(self, n_in, n_out, params):
        self.n_in, self.n_out = int(n_in), int(n_out)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(q, np.float32).ravel() for q in params]))
        self._h = C.c_void_p()
        _check(_lib.dg_mlp_create(self.n_in, 128, self.n_out, _f32p(flat), C.byref(self._h)), "dg_mlp_create")
        self.n_params = _lib.dg_mlp_param_count(self._h)
        assert self.n_params == flat.size

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.dg_mlp_destroy(h)
            self._h = C.c_void_p()

    def _unpack(self, flat):
        H, ni, no = 128, self.n_in, self.n_out
        sizes = [H * ni, H, H * H, H, no * H, no]
        shapes = [(H, ni), (H,), (H, H), (H,), (no, H), (no,)]
        out, o = [], 0
        for sz, sh in zip(sizes, shapes):
            out.append(flat[o:o + sz].reshape(sh))
            o += sz
        return out

    def params(self):
        flat = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.dg_mlp_get_params(self._h, _f32p(flat), flat.size), "dg_mlp_get_params")
        return self._unpack(flat)

    def forward(self, x, out=None, stream=None):
        import torch
        n = x.shape[0]
        if out is None:
            out = torch.empty((n, self.n_out), dtype=torch.float32, device=x.device)
        _check(_lib.dg_mlp_forward(self._h, _ptr(x, torch.float32), n, _ptr(out, torch.float32), _stream(stream)),
               "dg_mlp_forward")
        return out

    def grad(self, x, t, want_grads=False, want_loss=True, stream=None):
        """loss and (optionally) the packed gradient, which the next adam_step uses; with
        want_loss and want_grads False it only enqueues (returns None)"""
        import torch
        loss = C.c_double()
        g = np.zeros(self.n_params, dtype=np.float32) if want_grads else None
        _check(_lib.dg_mlp_grad(self._h, _ptr(x, torch.float32), _ptr(t, torch.float32), x.shape[0],
                                C.byref(loss) if want_loss else None, _f32p(g) if want_grads else None,
                                _stream(stream)), "dg_mlp_grad")
        if want_grads:
            return loss.value, self._unpack(g)
        return loss.value if want_loss else None

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.dg_mlp_adam_step(self._h, lr, beta1, beta2, eps, _stream(stream)), "dg_mlp_adam_step")


def affine_rows(x, mean, scale, stream=None):
    """x <- (x - mean) / scale row-wise, in place on the device; mean and scale (host arrays
    [width]) are staged on x's device for the call, which waits for the kernel so that the
    staged copies outlive it"""
    import torch
    m = torch.as_tensor(np.ascontiguousarray(mean, dtype=np.float32)).to(x.device)
    s = torch.as_tensor(np.ascontiguousarray(scale, dtype=np.float32)).to(x.device)
    st = _stream(stream)
    _check(_lib.dg_affine_rows(_ptr(x, torch.float32), x.shape[0], x.shape[1], _ptr(m, torch.float32),
                               _ptr(s, torch.float32), st), "dg_affine_rows")
    torch.cuda.synchronize(x.device)


def _warmstart_set(self, net, x_mean=None, x_scale=None, y_mean=None, y_scale=None):
    if net is None:
        _check(_lib.dg_warmstart_set(self._h, None, None, None, None, None), "dg_warmstart_set")
        self._ws_keep = None
        return
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (x_mean, x_scale, y_mean, y_scale)]
    _check(_lib.dg_warmstart_set(self._h, net._h, *[_f32p(a) for a in arrs]), "dg_warmstart_set")
    self._ws_keep = (net, arrs)


def _warmstart_record(self, x, y, capacity, every):
    import torch
    if capacity == 0:
        _check(_lib.dg_warmstart_record(self._h, None, None, 0, 1), "dg_warmstart_record")
        self._rec_keep = None
        return
    _check(_lib.dg_warmstart_record(self._h, _ptr(x, torch.float32), _ptr(y, torch.float32), capacity, every),
           "dg_warmstart_record")
    self._rec_keep = (x, y)


def _warmstart_recorded(self):
    c = C.c_int64()
    _check(_lib.dg_warmstart_recorded(self._h, C.byref(c)), "dg_warmstart_recorded")
    return c.value


Mesh.warmstart_set = _warmstart_set
Mesh.warmstart_record = _warmstart_record
Mesh.warmstart_recorded = _warmstart_recorded


def library_path():
    return _LIB_PATH


def version():
    return _lib.dg_version()
