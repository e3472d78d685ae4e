"""ctypes binding of ``libibproj.so`` (the C ABI in ``include/ibproj.h``).

Argument marshalling only: device arrays are float64/int32 torch tensors on
the current HIP device (contiguous), host arrays are numpy float64/int32, and
every call is enqueued on ``torch.cuda.current_stream()``. All arithmetic
runs in the library. Loading fails loudly when the library is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibproj.so")

IB_OK, IB_EINVAL, IB_EHIP, IB_ENOMEM, IB_ENOTCONV, IB_EGEOM, IB_ENAN = 0, -1, -2, -3, -4, -5, -6
IB_SPREAD_IRROT, IB_SPREAD_DELTA = 0, 1
MG_FP64, MG_MIXED = 0, 1
WS_ZERO, WS_PREV, WS_NN = 0, 1, 2
NN_CONV_AUTO, NN_CONV_DIRECT = 0, 1
FLOW_SWEEP_AUTO, FLOW_SWEEP_COLOUR = 0, 1

EXPORTS = ("ib_create", "ib_destroy", "ib_bin_markers", "ib_interp", "ib_spread",
           "ib_coefficients", "ib_density", "ib_rhs", "ib_update", "mg_setup", "mg_update_coeffs",
           "mg_update_density", "mg_solve",
           "mg_destroy", "mg_residual_norm", "mg_residual_norm_noalloc", "project_step", "ib_relocate_bspline",
           "ib_surface_geometry_3d", "ib_nn_param_count", "ib_nn_create", "ib_nn_destroy",
           "ib_nn_set_params", "ib_nn_get_params", "ib_nn_predict", "ib_nn_gradients",
           "ib_nn_train_step", "ib_nn_set_conv", "ib_flow_set_sweep",
           "ib_diagnostics", "ib_profile_enable", "ib_profile_reset", "ib_profile_read",
           "ib_advection", "ib_viscous", "ib_flow_create", "ib_flow_destroy", "ib_flow_reset",
           "ib_predict", "flow_step", "ib_axi_create", "ib_axi_destroy", "axi_project_step",
           "ib_axi_reset", "axi_predict", "axi_flow_step", "ib_enclosed_measure", "ib_mass_correct",
           "ib_indicator_create", "ib_indicator_destroy", "ib_indicator_solve", "ib_markers_add_delete", "ib_surface_lsq_3d", "ib_mesh_measure", "ib_mesh_mass_correct",
           "ib_last_error")

PROF_KINDS = ("smooth64", "smooth32", "restrict64", "restrict32", "prolong64", "prolong32", "resid",
              "sweep64", "sweep32", "sweep64_rho", "sweep_zero", "sweep_dots", "sweep_pro")


class IbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double)]


class Surface(C.Structure):
    _fields_ = [("n_markers", C.c_int), ("X", C.c_void_p), ("n_elems", C.c_int),
                ("elems", C.c_void_p), ("nrm", C.c_void_p), ("fs", C.c_void_p), ("ds", C.c_void_p)]


class MgOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int), ("n_coarsest", C.c_int),
                ("krylov", C.c_int), ("split_coarse", C.c_int)]


class MgStats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_res0", C.c_double), ("rel_res", C.c_double),
                ("res_hist", C.c_double * 128), ("true_checks", C.c_int)]

    def as_dict(self):
        return dict(cycles=self.cycles, rel_res0=self.rel_res0, rel_res=self.rel_res,
                    hist=list(self.res_hist[: min(self.cycles, 128)]), true_checks=self.true_checks)


class Params(C.Structure):
    _fields_ = [("rho_in", C.c_double), ("rho_out", C.c_double), ("sigma", C.c_double),
                ("dt", C.c_double), ("rtol", C.c_double), ("max_cycles", C.c_int),
                ("fixed_cycles", C.c_int), ("spread_mode", C.c_int), ("warm_start", C.c_int)]


class State(C.Structure):
    _fields_ = [("u_star", C.c_void_p * 3), ("p_prev", C.c_void_p), ("surf", Surface),
                ("X_host", C.c_void_p), ("nn", C.c_void_p), ("elems_host", C.c_void_p)]


class Outputs(C.Structure):
    _fields_ = [("p", C.c_void_p), ("u", C.c_void_p * 3), ("U", C.c_void_p), ("H", C.c_void_p),
                ("F", C.c_void_p * 3), ("fs_host", C.c_void_p), ("b", C.c_void_p),
                ("stats", MgStats), ("guess_accepted", C.c_int), ("guess_rel_res", C.c_double),
                ("prev_rel_res", C.c_double), ("guess_energy", C.c_double), ("prev_energy", C.c_double)]


class FlowStats(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("rel_res", C.c_double), ("first_step", C.c_int),
                ("frame_a", C.c_double), ("com", C.c_double), ("measure", C.c_double),
                ("mass_delta", C.c_double), ("checks", C.c_int)]

    def as_dict(self):
        return dict(sweeps=self.sweeps, rel_res=self.rel_res, first_step=self.first_step,
                    frame_a=self.frame_a, com=self.com, measure=self.measure,
                    mass_delta=self.mass_delta, checks=self.checks)


class FlowParams(C.Structure):
    _fields_ = [("mu_in", C.c_double), ("mu_out", C.c_double), ("rtol", C.c_double),
                ("max_sweeps", C.c_int), ("gravity", C.c_double), ("frame", C.c_int),
                ("c1", C.c_double), ("c2", C.c_double), ("mass_every", C.c_int),
                ("mass_target", C.c_double), ("indicator_density", C.c_int)]

    @staticmethod
    def from_dict(params):
        """mu_in, mu_out, pred_rtol, pred_max_sweeps; free fall: gravity, frame (bool),
        c1, c2 (0.1 each by default), mass_every, mass_target (0: the first step's);
        indicator_density (conventional scheme: properties follow eq ind_psn's I)."""
        fp = FlowParams()
        fp.mu_in = params.get("mu_in", 0.0)
        fp.mu_out = params.get("mu_out", 0.0)
        fp.rtol = params.get("pred_rtol", 1e-12)
        fp.max_sweeps = params.get("pred_max_sweeps", 200)
        fp.gravity = params.get("gravity", 0.0)
        fp.frame = 1 if params.get("frame", False) else 0
        fp.c1 = params.get("c1", 0.1)
        fp.c2 = params.get("c2", 0.1)
        fp.mass_every = int(params.get("mass_every", 0))
        fp.mass_target = params.get("mass_target", 0.0)
        fp.indicator_density = 1 if params.get("indicator_density", False) else 0
        return fp


class Diag(C.Structure):
    _fields_ = [("dP", C.c_double), ("tke", C.c_double), ("force_sum", C.c_double * 3),
                ("curl_max", C.c_double), ("f_max", C.c_double)]

    def as_dict(self):
        return dict(dP=self.dP, tke=self.tke, force_sum=list(self.force_sum),
                    curl_max=self.curl_max, f_max=self.f_max)


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (no GPU call is made here).

    torch is imported first: its HIP runtime is then the one the library binds
    to. Loaded the other way round, the process would hold two HIP runtimes
    (torch asks for its own copy by another file name) and the library's
    device allocations fail.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run python -m paper_1807_10504_amd.build)")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, f64 = C.c_void_p, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "ib_create": (i32, [P(Grid), i32, i32, P(vp)]),
        "ib_destroy": (None, [vp]),
        "ib_bin_markers": (i32, [vp, P(Surface), vp, vp, vp, vp]),
        "ib_interp": (i32, [vp, vp * 3, P(Surface), vp, vp]),
        "ib_spread": (i32, [vp, P(Surface), i32, vp * 3, vp, vp]),
        "ib_coefficients": (i32, [vp, vp, f64, f64, vp * 3, vp]),
        "ib_density": (i32, [vp, vp, f64, f64, vp, vp]),
        "ib_rhs": (i32, [vp, vp * 3, vp * 3, vp * 3, f64, vp, vp]),
        "ib_update": (i32, [vp, vp * 3, vp * 3, vp * 3, vp, f64, vp * 3, vp]),
        "mg_setup": (i32, [P(Grid), P(MgOpts), P(vp)]),
        "mg_update_coeffs": (i32, [vp, vp * 3, vp]),
        "mg_update_density": (i32, [vp, vp, vp]),
        "mg_solve": (i32, [vp, vp, vp, f64, i32, i32, P(MgStats), vp]),
        "mg_destroy": (None, [vp]),
        "mg_residual_norm": (i32, [vp, vp, vp, P(f64), vp]),
        "mg_residual_norm_noalloc": (i32, [P(Grid), vp, vp, vp, vp, vp]),
        "ib_nn_param_count": (i32, [i32]),
        "ib_nn_create": (i32, [P(Grid), P(vp)]),
        "ib_nn_destroy": (None, [vp]),
        "ib_nn_set_conv": (i32, [vp, i32]),
        "ib_flow_set_sweep": (i32, [vp, i32]),
        "ib_nn_set_params": (i32, [vp, vp, i32]),
        "ib_nn_get_params": (i32, [vp, vp, i32]),
        "ib_nn_predict": (i32, [vp, vp, vp, vp, f64, f64, vp, vp]),
        "ib_nn_gradients": (i32, [vp, vp, vp, vp, vp, f64, f64, vp, i32, P(f64), vp]),
        "ib_nn_train_step": (i32, [vp, i32, vp, vp, vp, vp, f64, f64, C.c_float, P(f64), vp]),
        "project_step": (i32, [vp, vp, P(Params), P(State), P(Outputs), vp]),
        "ib_relocate_bspline": (i32, [i32, vp, vp, f64, f64, f64, vp, vp, vp, vp]),
        "ib_surface_geometry_3d": (i32, [i32, vp, i32, vp, f64, vp, vp, vp]),
        "ib_diagnostics": (i32, [vp, vp, vp, vp, vp, P(Diag), vp]),
        "ib_profile_enable": (None, [i32]),
        "ib_profile_reset": (None, []),
        "ib_profile_read": (i32, [i32, P(C.c_longlong), P(f64)]),
        "ib_advection": (i32, [vp, vp * 3, vp, vp * 3, vp]),
        "ib_viscous": (i32, [vp, vp * 3, vp, vp * 3, vp]),
        "ib_flow_create": (i32, [P(Grid), P(vp)]),
        "ib_flow_destroy": (None, [vp]),
        "ib_flow_reset": (i32, [vp]),
        "ib_predict": (i32, [vp, vp * 3, vp, vp, vp, f64, f64, i32, vp * 3, P(FlowStats), vp]),
        "flow_step": (i32, [vp, vp, vp, P(Params), P(FlowParams), P(State), P(Outputs),
                            P(FlowStats), vp]),
        "ib_axi_create": (i32, [P(Grid), i32, P(vp)]),
        "ib_axi_destroy": (None, [vp]),
        "axi_project_step": (i32, [vp, vp, P(Params), P(State), P(Outputs), vp]),
        "ib_axi_reset": (i32, [vp]),
        "axi_predict": (i32, [vp, vp * 2, vp, vp, vp, f64, f64, i32, vp * 2, P(FlowStats), vp]),
        "axi_flow_step": (i32, [vp, vp, P(Params), P(FlowParams), P(State), P(Outputs), P(FlowStats), vp]),
        "ib_enclosed_measure": (i32, [i32, vp, f64, P(f64), P(f64)]),
        "ib_mass_correct": (i32, [i32, vp, vp, f64, f64, f64, f64, f64, P(f64)]),
        "ib_markers_add_delete": (i32, [i32, vp, f64, f64, f64, i32, vp, P(i32)]),
        "ib_surface_lsq_3d": (i32, [i32, vp, i32, vp, f64, vp, vp, vp, vp]),
        "ib_mesh_measure": (i32, [i32, vp, i32, vp, P(f64), P(f64)]),
        "ib_mesh_mass_correct": (i32, [i32, vp, vp, i32, vp, f64, f64, f64, f64, P(f64)]),
        "ib_indicator_create": (i32, [P(Grid), i32, P(vp)]),
        "ib_indicator_destroy": (None, [vp]),
        "ib_indicator_solve": (i32, [vp, vp, P(Surface), f64, i32, vp, P(MgStats), vp]),
        "ib_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != IB_OK:
        msg = _lib.ib_last_error().decode()
        raise IbError(rc, msg)


# ----------------------------------------------------------------------------
# marshalling helpers
def _dptr(t, dtype=None):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


def _hptr(a, dtype=np.float64):
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags["C_CONTIGUOUS"]):
        raise ValueError(f"expected a C-contiguous numpy {np.dtype(dtype)} array")
    return a.ctypes.data


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _vec3(ts, dtype):
    import torch
    arr = (C.c_void_p * 3)()
    for e, t in enumerate(ts):
        arr[e] = _dptr(t, dtype)
    return arr


def make_grid(dim, n, h) -> Grid:
    g = Grid()
    g.dim = dim
    for e in range(3):
        g.n[e] = int(n[e]) if e < len(n) else 1
    g.h = float(h)
    return g


def make_surface(X, elems=None, nrm=None, fs=None, ds=None) -> Surface:
    import torch
    s = Surface()
    s.n_markers = int(X.shape[0])
    s.X = _dptr(X, torch.float64)
    s.n_elems = 0 if elems is None else int(elems.shape[0])
    s.elems = _dptr(elems, torch.int32)
    s.nrm = _dptr(nrm, torch.float64)
    s.fs = _dptr(fs, torch.float64)
    s.ds = _dptr(ds, torch.float64)
    # the structure holds raw device pointers: keep the tensors alive with it
    s._keep = (X, elems, nrm, fs, ds)
    return s


# ----------------------------------------------------------------------------
class Context:
    """Workspace for binning, spreading and projection steps on one grid."""

    def __init__(self, dim, n, h, max_markers, max_elems=0):
        import torch
        self.lib = load()
        self.dim, self.n, self.h = dim, tuple(n[:dim]), float(h)
        self.grid = make_grid(dim, n, h)
        self.ptr = C.c_void_p()
        _check(self.lib.ib_create(C.byref(self.grid), int(max_markers), int(max_elems),
                                  C.byref(self.ptr)))
        self.shape = tuple(reversed(self.n))

    def close(self):
        if self.ptr:
            self.lib.ib_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_tiles(self):
        t = 1
        for e in range(self.dim):
            t *= self.n[e] // 4
        return t

    def bin_markers(self, surf: Surface):
        import torch
        n = surf.n_markers
        key = torch.empty(n, dtype=torch.int32, device="cuda")
        order = torch.empty(n, dtype=torch.int32, device="cuda")
        start = torch.empty(self.n_tiles + 1, dtype=torch.int32, device="cuda")
        _check(self.lib.ib_bin_markers(self.ptr, C.byref(surf), key.data_ptr(), order.data_ptr(),
                                       start.data_ptr(), _stream()))
        return key, order, start

    def interp(self, u, surf: Surface, U=None):
        import torch
        if U is None:
            U = torch.empty((surf.n_markers, self.dim), dtype=torch.float64, device="cuda")
        _check(self.lib.ib_interp(self.ptr, _vec3(u, torch.float64), C.byref(surf),
                                  _dptr(U, torch.float64), _stream()))
        return U

    def spread(self, surf: Surface, mode=IB_SPREAD_IRROT, F=None, H=None, want_H=True):
        import torch
        if F is None:
            F = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        if H is None and (want_H or mode == IB_SPREAD_IRROT):
            H = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _check(self.lib.ib_spread(self.ptr, C.byref(surf), mode, _vec3(F, torch.float64),
                                  _dptr(H, torch.float64), _stream()))
        return F, H

    def coefficients(self, H, rho_in, rho_out, beta=None):
        import torch
        if beta is None:
            beta = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        _check(self.lib.ib_coefficients(self.ptr, _dptr(H, torch.float64), rho_in, rho_out,
                                        _vec3(beta, torch.float64), _stream()))
        return beta

    def density(self, H, rho_in, rho_out, rho=None):
        import torch
        if rho is None:
            rho = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _check(self.lib.ib_density(self.ptr, _dptr(H, torch.float64), rho_in, rho_out,
                                   _dptr(rho, torch.float64), _stream()))
        return rho

    def rhs(self, u_star, F, beta, dt, b=None):
        import torch
        if b is None:
            b = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _check(self.lib.ib_rhs(self.ptr, _vec3(u_star, torch.float64), _vec3(F, torch.float64),
                               _vec3(beta, torch.float64), dt, _dptr(b, torch.float64), _stream()))
        return b

    def update(self, u_star, F, beta, p, dt, u_new=None):
        import torch
        if u_new is None:
            u_new = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        _check(self.lib.ib_update(self.ptr, _vec3(u_star, torch.float64), _vec3(F, torch.float64),
                                  _vec3(beta, torch.float64), _dptr(p, torch.float64), dt,
                                  _vec3(u_new, torch.float64), _stream()))
        return u_new

    def diagnostics(self, p=None, H=None, u=None, F=None):
        import torch
        d = Diag()
        ua = _vec3(u, torch.float64) if u is not None else None
        Fa = _vec3(F, torch.float64) if F is not None else None
        _check(self.lib.ib_diagnostics(self.ptr, _dptr(p, torch.float64), _dptr(H, torch.float64),
                                       C.addressof(ua) if ua is not None else None,
                                       C.addressof(Fa) if Fa is not None else None,
                                       C.byref(d), _stream()))
        return d.as_dict()

    def advection(self, u, rho, A=None):
        """C(u) of eq ad_bf (per face component)."""
        import torch
        if A is None:
            A = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        _check(self.lib.ib_advection(self.ptr, _vec3(u, torch.float64), _dptr(rho, torch.float64),
                                     _vec3(A, torch.float64), _stream()))
        return A

    def viscous(self, u, mu, V=None):
        """D u of eq cr_ni (per face component)."""
        import torch
        if V is None:
            V = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        _check(self.lib.ib_viscous(self.ptr, _vec3(u, torch.float64), _dptr(mu, torch.float64),
                                   _vec3(V, torch.float64), _stream()))
        return V

    @staticmethod
    def _params(params, p_prev):
        prm = Params()
        prm.rho_in = params["rho_in"]
        prm.rho_out = params["rho_out"]
        prm.sigma = params.get("sigma", 1.0)
        prm.dt = params["dt"]
        prm.rtol = params.get("rtol", 1e-10)
        prm.max_cycles = params.get("max_cycles", 100)
        prm.fixed_cycles = params.get("fixed_cycles", 0)
        prm.spread_mode = params.get("spread_mode", IB_SPREAD_IRROT)
        prm.warm_start = params.get("warm_start", WS_PREV if p_prev is not None else WS_ZERO)
        return prm

    def _outputs(self, out, nm):
        import torch
        if out is None:
            out = {}
        o = Outputs()
        shape = self.shape
        dev = "cuda"
        out.setdefault("p", torch.empty(shape, dtype=torch.float64, device=dev))
        out.setdefault("u", [torch.empty(shape, dtype=torch.float64, device=dev) for _ in range(self.dim)])
        out.setdefault("U", torch.empty((nm, self.dim), dtype=torch.float64, device=dev))
        o.p = _dptr(out["p"], torch.float64)
        o.u = _vec3(out["u"], torch.float64)
        o.U = _dptr(out["U"], torch.float64)
        o.H = _dptr(out.get("H"), torch.float64)
        o.F = _vec3(out["F"], torch.float64) if out.get("F") is not None else (C.c_void_p * 3)()
        fs_host = out.get("fs_host")
        o.fs_host = _hptr(fs_host) if fs_host is not None else None
        o.b = _dptr(out.get("b"), torch.float64)
        return out, o

    def project_step(self, mg: "Multigrid", params: dict, u_star, p_prev=None, surf=None,
                     X_host=None, n_markers=None, out=None, nn: "Network" = None):
        """One projection step. 2D: X_host (numpy, N x 2) is advanced and relocated in
        place; 3D: surf is the static surface. Returns the outputs dict."""
        import torch
        prm = self._params(params, p_prev)
        st = State()
        st.u_star = _vec3(u_star, torch.float64)
        st.p_prev = _dptr(p_prev, torch.float64)
        if self.dim == 2:
            st.surf = Surface()
            st.surf.n_markers = int(X_host.shape[0])
            st.X_host = _hptr(X_host)
            nm = int(X_host.shape[0])
        else:
            st.surf = surf
            st.X_host = None
            nm = surf.n_markers
        st.nn = nn.ptr if nn is not None else None
        out, o = self._outputs(out, nm)
        rc = self.lib.project_step(self.ptr, mg.ptr, C.byref(prm), C.byref(st), C.byref(o), _stream())
        out["stats"] = o.stats.as_dict()
        out["guess"] = dict(accepted=o.guess_accepted, rel_res=o.guess_rel_res,
                            prev_rel_res=o.prev_rel_res,
                            energy=o.guess_energy, prev_energy=o.prev_energy)
        if rc == IB_ENOTCONV and params.get("allow_notconv", False):
            return out
        _check(rc)
        return out

    def flow_step(self, mg: "Multigrid", flow: "Flow", params: dict, u, X_host, p_prev=None,
                  out=None, tris=None):
        """One step of the full method: markers advanced with u^n (X_host, numpy N x dim,
        updated in place; 3D: the vertices of the surface whose triangles `tris`,
        numpy int32 M x 3, stay fixed), H and force of the new markers, predictor
        (params: mu_in, mu_out, pred_rtol, pred_max_sweeps; free fall: gravity, frame,
        c1, c2, mass_every -- FlowParams.from_dict), projection. Returns the outputs dict
        with 'stats' (multigrid) and 'flow' (predictor)."""
        import torch
        prm = self._params(params, p_prev)
        fp = FlowParams.from_dict(params)
        st = State()
        st.u_star = _vec3(u, torch.float64)
        st.p_prev = _dptr(p_prev, torch.float64)
        st.surf = Surface()
        st.surf.n_markers = int(X_host.shape[0])
        st.X_host = _hptr(X_host)
        st.nn = None
        st.elems_host = None
        if self.dim == 3:
            if tris is None:
                raise ValueError("a 3D flow step needs the surface's triangles")
            tris = np.ascontiguousarray(tris, dtype=np.int32)
            cached = getattr(self, "_tris_host", None)
            if cached is None or cached.shape != tris.shape or not np.array_equal(cached, tris):
                self._tris_host = tris.copy()
                self._tris_dev = torch.from_numpy(self._tris_host).cuda()
            st.surf.n_elems = int(tris.shape[0])
            st.surf.elems = self._tris_dev.data_ptr()
            st.elems_host = _hptr(self._tris_host, np.int32)
        out, o = self._outputs(out, int(X_host.shape[0]))
        fs = FlowStats()
        rc = self.lib.flow_step(self.ptr, flow.ptr, mg.ptr, C.byref(prm), C.byref(fp), C.byref(st),
                                C.byref(o), C.byref(fs), _stream())
        out["stats"] = o.stats.as_dict()
        out["flow"] = fs.as_dict()
        _check(rc)
        return out


class Flow:
    """Momentum predictor state (Adams-Bashforth history, previous H, workspace)."""

    def __init__(self, dim, n, h):
        self.lib = load()
        self.dim = dim
        self.shape = tuple(reversed(tuple(n[:dim])))
        self.grid = make_grid(dim, n, h)
        self.ptr = C.c_void_p()
        _check(self.lib.ib_flow_create(C.byref(self.grid), C.byref(self.ptr)))

    def close(self):
        if self.ptr:
            self.lib.ib_flow_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(self.lib.ib_flow_reset(self.ptr))

    def set_sweep(self, kind):
        """FLOW_SWEEP_AUTO (single-pass sweep where the grid allows) or FLOW_SWEEP_COLOUR."""
        _check(self.lib.ib_flow_set_sweep(self.ptr, int(kind)))

    def predict(self, u, rho_n, rho_np1, mu, dt, rtol=1e-12, max_sweeps=200, u_star=None):
        """u* of eq ns1_new; returns (u_star, stats dict)."""
        import torch
        if u_star is None:
            u_star = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(self.dim)]
        fs = FlowStats()
        _check(self.lib.ib_predict(self.ptr, _vec3(u, torch.float64), _dptr(rho_n, torch.float64),
                                   _dptr(rho_np1, torch.float64), _dptr(mu, torch.float64), dt, rtol,
                                   int(max_sweeps), _vec3(u_star, torch.float64), C.byref(fs), _stream()))
        return u_star, fs.as_dict()


class Axisym:
    """Axisymmetric projection on the meridian half plane (nr x nz cells, spacing h).
    Markers are the meridian curve mirrored about the axis, closed and counter-
    clockwise, in a doubled plane whose axis is x = nr h."""

    def __init__(self, nr, nz, h, max_markers):
        self.lib = load()
        self.nr, self.nz, self.h = nr, nz, float(h)
        self.dim = 2
        self.shape = (nz, nr)
        self.grid = make_grid(2, (nr, nz), h)
        self.ptr = C.c_void_p()
        _check(self.lib.ib_axi_create(C.byref(self.grid), int(max_markers), C.byref(self.ptr)))

    def close(self):
        if self.ptr:
            self.lib.ib_axi_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def project_step(self, mg: "Multigrid", params: dict, u_star, X_host, p_prev=None, out=None,
                     nn: "Network" = None):
        """One axisymmetric projection step; X_host (numpy, N x 2) is advanced and
        relocated in place. Returns the outputs dict (half-plane fields)."""
        import torch
        prm = Context._params(params, p_prev)
        st = State()
        st.u_star = _vec3(u_star, torch.float64)
        st.p_prev = _dptr(p_prev, torch.float64)
        st.surf = Surface()
        st.surf.n_markers = int(X_host.shape[0])
        st.X_host = _hptr(X_host)
        st.nn = nn.ptr if nn is not None else None
        out, o = Context._outputs(self, out, int(X_host.shape[0]))
        rc = self.lib.axi_project_step(self.ptr, mg.ptr, C.byref(prm), C.byref(st), C.byref(o), _stream())
        out["stats"] = o.stats.as_dict()
        out["guess"] = dict(accepted=o.guess_accepted, rel_res=o.guess_rel_res, prev_rel_res=o.prev_rel_res,
                            energy=o.guess_energy, prev_energy=o.prev_energy)
        _check(rc)
        return out

    def reset(self):
        _check(self.lib.ib_axi_reset(self.ptr))

    def predict(self, u, rho_n, rho_np1, mu, dt, rtol=1e-12, max_sweeps=200, u_star=None):
        """u* of the meridian-plane predictor; returns (u_star, stats dict)."""
        import torch
        if u_star is None:
            u_star = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(2)]
        fs = FlowStats()
        uv = (C.c_void_p * 2)(*[_dptr(x, torch.float64) for x in u])
        sv = (C.c_void_p * 2)(*[_dptr(x, torch.float64) for x in u_star])
        _check(self.lib.axi_predict(self.ptr, uv, _dptr(rho_n, torch.float64), _dptr(rho_np1, torch.float64),
                                    _dptr(mu, torch.float64), dt, rtol, int(max_sweeps), sv, C.byref(fs),
                                    _stream()))
        return u_star, fs.as_dict()

    def flow_step(self, mg: "Multigrid", params: dict, u, X_host, p_prev=None, out=None,
                  nn: "Network" = None):
        """One full axisymmetric step (params as Context.flow_step)."""
        import torch
        prm = Context._params(params, p_prev)
        fp = FlowParams.from_dict(params)
        st = State()
        st.u_star = _vec3(u, torch.float64)
        st.p_prev = _dptr(p_prev, torch.float64)
        st.surf = Surface()
        st.surf.n_markers = int(X_host.shape[0])
        st.X_host = _hptr(X_host)
        st.nn = nn.ptr if nn is not None else None
        out, o = Context._outputs(self, out, int(X_host.shape[0]))
        fs = FlowStats()
        rc = self.lib.axi_flow_step(self.ptr, mg.ptr, C.byref(prm), C.byref(fp), C.byref(st), C.byref(o),
                                    C.byref(fs), _stream())
        out["stats"] = o.stats.as_dict()
        out["guess"] = dict(accepted=o.guess_accepted, rel_res=o.guess_rel_res, prev_rel_res=o.prev_rel_res,
                            energy=o.guess_energy, prev_energy=o.prev_energy)
        out["flow"] = fs.as_dict()
        _check(rc)
        return out


class Indicator:
    """Indicator function of the conventional scheme (eq ind_psn) on a 2D grid."""

    def __init__(self, n, h, max_markers):
        self.lib = load()
        self.grid = make_grid(2, n, h)
        self.shape = tuple(reversed(tuple(n[:2])))
        self.max_markers = int(max_markers)
        self.ptr = C.c_void_p()
        _check(self.lib.ib_indicator_create(C.byref(self.grid), self.max_markers, C.byref(self.ptr)))

    def close(self):
        if self.ptr:
            self.lib.ib_indicator_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, ctx: "Context", X, nrm, ds, rtol=1e-12, max_cycles=100, I=None):
        """I for the markers X (device tensor N x 2), unit normals nrm (N x 2, toward
        the drop) and arc elements ds (N); returns (I, stats dict)."""
        import torch
        if I is None:
            I = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        s = Surface()
        s.n_markers = int(X.shape[0])
        s.X = _dptr(X, torch.float64)
        s.nrm = _dptr(nrm, torch.float64)
        s.ds = _dptr(ds, torch.float64)
        st = MgStats()
        rc = self.lib.ib_indicator_solve(ctx.ptr, self.ptr, C.byref(s), float(rtol), int(max_cycles),
                                         _dptr(I, torch.float64), C.byref(st), _stream())
        _check(rc)
        return I, st.as_dict()


class Multigrid:
    def __init__(self, dim, n, h, precision=MG_FP64, nu1=2, nu2=2, n_coarsest=4, krylov=0,
                 split_coarse=0):
        self.lib = load()
        self.grid = make_grid(dim, n, h)
        o = MgOpts()
        o.precision, o.nu1, o.nu2, o.n_coarsest = precision, nu1, nu2, n_coarsest
        o.krylov = krylov
        o.split_coarse = split_coarse
        self.opts = o
        self.dim = dim
        self.ptr = C.c_void_p()
        _check(self.lib.mg_setup(C.byref(self.grid), C.byref(o), C.byref(self.ptr)))

    def close(self):
        if self.ptr:
            self.lib.mg_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_coeffs(self, beta):
        import torch
        self._beta = list(beta)  # keep the arrays alive while the handle refers to them
        _check(self.lib.mg_update_coeffs(self.ptr, _vec3(beta, torch.float64), _stream()))

    def update_density(self, rho):
        import torch
        self._beta = [rho]  # keep the array alive while the handle refers to it
        _check(self.lib.mg_update_density(self.ptr, _dptr(rho, torch.float64), _stream()))

    def residual_norm(self, b, p):
        import torch
        r = C.c_double()
        _check(self.lib.mg_residual_norm(self.ptr, _dptr(b, torch.float64), _dptr(p, torch.float64),
                                         C.byref(r), _stream()))
        return r.value

    def solve(self, b, p, rtol=1e-10, max_cycles=100, fixed_cycles=0, allow_notconv=False):
        import torch
        st = MgStats()
        rc = self.lib.mg_solve(self.ptr, _dptr(b, torch.float64), _dptr(p, torch.float64), rtol,
                               max_cycles, fixed_cycles, C.byref(st), _stream())
        if not (rc == IB_ENOTCONV and allow_notconv):
            _check(rc)
        return st.as_dict()


# ----------------------------------------------------------------------------
class Network:
    """The learned warm start: bfloat16 convolutional network on the matrix cores
    (2D with n = (nx, ny), 3D with n = (nx, ny, nz))."""

    def __init__(self, n, h):
        self.lib = load()
        self.dim = len(n)
        self.grid = make_grid(self.dim, n, h)
        self.ptr = C.c_void_p()
        _check(self.lib.ib_nn_create(C.byref(self.grid), C.byref(self.ptr)))
        self.count = self.lib.ib_nn_param_count(self.dim)

    def close(self):
        if self.ptr:
            self.lib.ib_nn_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_conv(self, kind):
        """NN_CONV_AUTO (tiled kernel where the grid allows) or NN_CONV_DIRECT."""
        _check(self.lib.ib_nn_set_conv(self.ptr, int(kind)))

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(self.lib.ib_nn_set_params(self.ptr, flat.ctypes.data, flat.size))

    def get_params(self):
        out = np.empty(self.count, dtype=np.float32)
        _check(self.lib.ib_nn_get_params(self.ptr, out.ctypes.data, out.size))
        return out

    def predict(self, b, H, p_prev, rho_in, rho_out, p0=None):
        import torch
        if p0 is None:
            p0 = torch.empty_like(b)
        _check(self.lib.ib_nn_predict(self.ptr, _dptr(b, torch.float64), _dptr(H, torch.float64),
                                      _dptr(p_prev, torch.float64), rho_in, rho_out,
                                      _dptr(p0, torch.float64), _stream()))
        return p0

    def gradients(self, b, H, p_prev, p, rho_in, rho_out):
        import torch
        g = np.empty(self.count, dtype=np.float32)
        loss = C.c_double()
        _check(self.lib.ib_nn_gradients(self.ptr, _dptr(b, torch.float64), _dptr(H, torch.float64),
                                        _dptr(p_prev, torch.float64), _dptr(p, torch.float64), rho_in,
                                        rho_out, g.ctypes.data, g.size, C.byref(loss), _stream()))
        return loss.value, g

    def train_step(self, samples, rho_in, rho_out, lr):
        """samples: list of (b, H, p_prev, p) device tensors. Returns the mean loss."""
        import torch
        n = len(samples)
        arr = [(C.c_void_p * n)() for _ in range(4)]
        for i, smp in enumerate(samples):
            for j in range(4):
                arr[j][i] = _dptr(smp[j], torch.float64)
        loss = C.c_double()
        _check(self.lib.ib_nn_train_step(self.ptr, n, arr[0], arr[1], arr[2], arr[3], rho_in, rho_out,
                                         C.c_float(lr), C.byref(loss), _stream()))
        return loss.value


def flatten_params(params):
    """Oracle parameter list [[W, b], ...] -> the ABI's flat float32 layout."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflatten_params(flat, channels=(3, 32, 32, 32, 32, 32, 1), dim=2):
    out, o = [], 0
    for l in range(6):
        ci, co = channels[l], channels[l + 1]
        nW = co * ci * 3 ** dim
        W = flat[o:o + nW].reshape((co, ci) + (3,) * dim).astype(np.float64)
        o += nW
        b = flat[o:o + co].astype(np.float64)
        o += co
        out.append([W, b])
    return out


# ----------------------------------------------------------------------------
# kernel timing
def residual_norm_noalloc(dim, n, h, rho, b, p, rel):
    """||b - A p|| / ||b|| for the face coefficients 2 / (rho_c + rho_{c-e_d}),
    written to the one-element float64 device tensor `rel` in stream order;
    no handle, no allocation, no host sync (mg_residual_norm_noalloc)."""
    import torch
    lib = load()
    g = make_grid(dim, n, h)
    _check(lib.mg_residual_norm_noalloc(C.byref(g), _dptr(rho, torch.float64), _dptr(b, torch.float64),
                                        _dptr(p, torch.float64), _dptr(rel, torch.float64), _stream()))
    return rel


def profile_enable(on=True):
    load().ib_profile_enable(1 if on else 0)


def profile_reset():
    load().ib_profile_reset()


def profile_read():
    """{kind: (launches, total_ms)} for the finest-level multigrid kernels."""
    lib = load()
    out = {}
    for k, name in enumerate(PROF_KINDS):
        n = C.c_longlong()
        ms = C.c_double()
        _check(lib.ib_profile_read(k, C.byref(n), C.byref(ms)))
        out[name] = (int(n.value), float(ms.value))
    return out


# ----------------------------------------------------------------------------
# host FP64 interface geometry
def relocate_bspline(X, U, dt, h, sigma):
    lib = load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = X.shape[0]
    Xo = np.empty_like(X)
    fs = np.empty(n)
    ds = np.empty(n)
    nrm = np.empty_like(X)
    _check(lib.ib_relocate_bspline(n, _hptr(X), _hptr(U), dt, h, sigma, _hptr(Xo), _hptr(fs),
                                   _hptr(ds), _hptr(nrm)))
    return Xo, fs, ds, nrm


def enclosed_measure(X, axis_x=None):
    """(enclosed area, vertical centroid) of the closed polygon X, or (volume of
    revolution about x = axis_x, axial centroid) of the mirrored meridian curve."""
    lib = load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    v, c = C.c_double(), C.c_double()
    _check(lib.ib_enclosed_measure(X.shape[0], _hptr(X), float("nan") if axis_x is None else float(axis_x),
                                   C.byref(v), C.byref(c)))
    return v.value, c.value


def mass_correct(X, nrm, target, axis_x=None, h=1.0, trigger=1e-6, tol=1e-12):
    """Markers moved along their normals back to the enclosed measure `target`;
    returns (X corrected, displacement)."""
    lib = load()
    Xc = np.array(X, dtype=np.float64, order="C")
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    d = C.c_double()
    _check(lib.ib_mass_correct(Xc.shape[0], _hptr(Xc), _hptr(nrm), float(target),
                               float("nan") if axis_x is None else float(axis_x), float(h), float(trigger),
                               float(tol), C.byref(d)))
    return Xc, d.value


def mesh_measure(V, T):
    """(volume enclosed by the closed mesh, y of its centroid)."""
    lib = load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    v, c = C.c_double(), C.c_double()
    _check(lib.ib_mesh_measure(V.shape[0], _hptr(V), T.shape[0], _hptr(T, np.int32), C.byref(v), C.byref(c)))
    return v.value, c.value


def mesh_mass_correct(V, nrm, T, target, h, trigger=1e-6, tol=1e-12):
    """Mesh vertices moved along their normals back to the enclosed volume `target`;
    returns (V corrected, displacement)."""
    lib = load()
    Vc = np.array(V, dtype=np.float64, order="C")
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    d = C.c_double()
    _check(lib.ib_mesh_mass_correct(Vc.shape[0], _hptr(Vc), _hptr(nrm), T.shape[0], _hptr(T, np.int32),
                                    float(target), float(h), float(trigger), float(tol), C.byref(d)))
    return Vc, d.value


def markers_add_delete(X, h, lo=0.5, hi=1.5):
    """Conventional marker deletion (closer than lo h) and midpoint addition (gaps
    beyond hi h) on the closed curve X; returns the new curve."""
    lib = load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    cap = 2 * X.shape[0]
    out = np.empty((cap, 2))
    m = C.c_int()
    _check(lib.ib_markers_add_delete(X.shape[0], _hptr(X), float(h), float(lo), float(hi), cap, _hptr(out),
                                     C.byref(m)))
    return out[: m.value].copy()


def surface_lsq_3d(V, T, sigma):
    """Local least-squares reconstruction of a closed triangulated surface: returns
    (V', fs, ds, nrm)."""
    lib = load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    Vo = np.empty_like(V)
    fs = np.empty(V.shape[0])
    ds = np.empty(V.shape[0])
    nrm = np.empty_like(V)
    _check(lib.ib_surface_lsq_3d(V.shape[0], _hptr(V), T.shape[0], _hptr(T, np.int32), float(sigma), _hptr(Vo), _hptr(fs),
                                 _hptr(ds), _hptr(nrm)))
    return Vo, fs, ds, nrm


def surface_geometry_3d(V, T, sigma):
    lib = load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    nv = V.shape[0]
    fs = np.empty(nv)
    ds = np.empty(nv)
    nrm = np.empty_like(V)
    _check(lib.ib_surface_geometry_3d(nv, _hptr(V), T.shape[0], _hptr(T, np.int32), sigma,
                                      _hptr(fs), _hptr(ds), _hptr(nrm)))
    return fs, ds, nrm
