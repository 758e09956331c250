"""Python binding of the MI355X pipe-flow time-step library (libopf.so).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (the workspace and state tensors)
and the HIP stream.  The binding fails loudly when the library is missing;
there is no CPU fallback.

Names follow include/opf.h; see that header for layouts and semantics.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopf.so")

OPF_OK, OPF_E_INVALID, OPF_E_NOMEM, OPF_E_HIP, OPF_E_UNSUPPORTED, OPF_E_NUMERIC, OPF_E_STATE = (
    0, -1, -2, -3, -4, -5, -6)
OPF_FP64, OPF_MIXED = 0, 1
OPF_SOLVE_PRED, OPF_SOLVE_CORR, OPF_SOLVE_RAW = 0, 1, 2

EXPORTS = ["opf_default_params", "opf_tables", "opf_workspace_size", "opf_create", "opf_destroy",
           "opf_get_nodes", "opf_set_state", "opf_get_state", "opf_step", "opf_nonlinear",
           "opf_vorticity", "opf_radial_solve", "opf_newton_residual", "opf_profile_steps",
           "opf_vec_dot", "opf_vec_axpby", "opf_nk_workspace_size", "opf_nk_solve",
           "opf_diagnostics", "opf_probe_pairs", "opf_mlp_default_config", "opf_mlp_workspace_size", "opf_mlp_create",
           "opf_mlp_destroy", "opf_mlp_dims", "opf_mlp_set_params", "opf_mlp_get_params",
           "opf_mlp_forward", "opf_mlp_gradient", "opf_mlp_train", "opf_mlp_pair_gradient",
           "opf_mlp_train_pairs", "opf_mlp_factors", "opf_precondition", "opf_mlp_last_error", "opf_ensemble_workspace_size", "opf_ensemble_create",
           "opf_ensemble_destroy", "opf_ensemble_member", "opf_ensemble_step", "opf_ensemble_tune",
           "opf_ensemble_tiles", "opf_autotune", "opf_tile_cache_write", "opf_tile_cache_read",
           "opf_probe_pairs_noalloc",
           "opf_ensemble_last_error", "opf_probe_pairs_ensemble", "opf_set_dt", "opf_pc_difference",
           "opf_step_adaptive", "opf_hookstep_solve", "opf_arnoldi_workspace_size", "opf_arnoldi",
           "opf_hessenberg_eigvals", "opf_set_rotation", "opf_shoot_workspace_size", "opf_shoot_solve", "opf_set_wall_velocity",
           "opf_status_string", "opf_last_error"]


class opf_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
                ("mp", ctypes.c_int32), ("stencil", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("Re", ctypes.c_double), ("dt", ctypes.c_double),
                ("c", ctypes.c_double),
                ("n_corr", ctypes.c_int32), ("fixed_flux", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("nonlinear", ctypes.c_int32),
                ("r_nodes", ctypes.c_void_p)]


class opf_diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("E", "I", "D", "tau_w", "flux", "beta", "E_lam", "I_lam", "D_lam", "g_norm", "div_max",
                 "cfl")]


class opf_dt_control(ctypes.Structure):
    _fields_ = [("courant", ctypes.c_double), ("pc_tol", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("grow", ctypes.c_double), ("check_every", ctypes.c_int32)]


class opf_dt_report(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("checks", ctypes.c_int32), ("changes", ctypes.c_int32),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("pc_diff", ctypes.c_double), ("rebuild_ms", ctypes.c_double)]


class opf_arnoldi_report(ctypes.Structure):
    _fields_ = [("products", ctypes.c_int32), ("converged", ctypes.c_int32), ("checks", ctypes.c_int32)]


class opf_shoot_opts(ctypes.Structure):
    _fields_ = [("sections", ctypes.c_int32), ("steps", ctypes.c_int32), ("free_T", ctypes.c_int32),
                ("free_s", ctypes.c_int32), ("gmres_m", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("tol", ctypes.c_double), ("gmres_tol", ctypes.c_double), ("fd_eps", ctypes.c_double),
                ("tr_delta0", ctypes.c_double), ("tr_delta_max", ctypes.c_double), ("max_hook", ctypes.c_int32)]


class opf_shoot_report(ctypes.Structure):
    _fields_ = [("newton_iterations", ctypes.c_int32), ("products", ctypes.c_int32),
                ("residual_evals", ctypes.c_int32), ("hook_trials", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("stalled", ctypes.c_int32), ("residual", ctypes.c_double),
                ("residual_history", ctypes.c_double * 32), ("T", ctypes.c_double), ("shift", ctypes.c_double),
                ("tr_delta", ctypes.c_double)]


class opf_nk_opts(ctypes.Structure):
    _fields_ = [("gmres_m", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_jvps", ctypes.c_int32), ("tol", ctypes.c_double),
                ("gmres_tol", ctypes.c_double), ("fd_eps", ctypes.c_double),
                ("precond", ctypes.c_void_p), ("record_dev", ctypes.c_void_p),
                ("record_capacity", ctypes.c_int32), ("hookstep", ctypes.c_int32),
                ("tr_delta0", ctypes.c_double), ("tr_delta_max", ctypes.c_double),
                ("max_hook", ctypes.c_int32), ("free_speed", ctypes.c_int32),
                ("no_fallback", ctypes.c_int32), ("speed_freeze", ctypes.c_double)]


class opf_nk_report(ctypes.Structure):
    _fields_ = [("newton_iterations", ctypes.c_int32), ("gmres_iterations", ctypes.c_int32),
                ("jvps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual", ctypes.c_double), ("residual_history", ctypes.c_double * 32),
                ("recorded", ctypes.c_int32), ("precond_applies", ctypes.c_int32),
                ("residual_evals", ctypes.c_int32), ("hook_trials", ctypes.c_int32),
                ("stalled", ctypes.c_int32), ("tr_delta", ctypes.c_double),
                ("speed", ctypes.c_double), ("frozen_steps", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32)]


class opf_mlp_config(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("layers", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("max_rows", ctypes.c_int32), ("seed", ctypes.c_uint64), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float), ("lr_final", ctypes.c_float)]


class opf_tiles(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("K", ctypes.c_int32), ("mp", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("members", ctypes.c_int32), ("gm", ctypes.c_int32),
                ("tz", ctypes.c_int32), ("ztile", ctypes.c_int32), ("us_per_step", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class OpfError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"opf status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path=LIB_PATH):
    """Load libopf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OpfError(OPF_E_UNSUPPORTED, f"{path} not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "opf_default_params": ([P(opf_params)], i32),
        "opf_tables": ([P(opf_params), vp, vp, vp, vp, vp], i32),
        "opf_workspace_size": ([P(opf_params), P(ctypes.c_size_t)], i32),
        "opf_create": ([P(opf_params), vp, ctypes.c_size_t, vp, P(vp)], i32),
        "opf_destroy": ([vp], i32),
        "opf_get_nodes": ([vp, P(ctypes.c_double)], i32),
        "opf_set_state": ([vp, vp], i32),
        "opf_get_state": ([vp, vp], i32),
        "opf_step": ([vp, i32], i32),
        "opf_nonlinear": ([vp, vp, vp], i32),
        "opf_vorticity": ([vp, vp, vp], i32),
        "opf_radial_solve": ([vp, i32, vp, vp, vp], i32),
        "opf_newton_residual": ([vp, vp, dbl, dbl, vp, P(ctypes.c_double)], i32),
        "opf_profile_steps": ([vp, i32, P(ctypes.c_double), P(ctypes.c_int32)], i32),
        "opf_vec_dot": ([vp, vp, vp, P(ctypes.c_double)], i32),
        "opf_vec_axpby": ([vp, dbl, vp, dbl, vp], i32),
        "opf_nk_workspace_size": ([vp, i32, i32, P(ctypes.c_size_t)], i32),
        "opf_nk_solve": ([vp, vp, dbl, P(dbl), P(opf_nk_opts), vp, ctypes.c_size_t, P(opf_nk_report)], i32),
        "opf_diagnostics": ([vp, P(opf_diag)], i32),
        "opf_probe_pairs": ([vp, vp, dbl, dbl, i32, ctypes.c_uint64, dbl, vp, vp], i32),
        "opf_probe_pairs_noalloc": ([vp, vp, dbl, dbl, i32, ctypes.c_uint64, dbl, vp], i32),
        "opf_mlp_default_config": ([P(opf_mlp_config)], i32),
        "opf_mlp_workspace_size": ([vp, P(opf_mlp_config), P(ctypes.c_size_t)], i32),
        "opf_mlp_create": ([vp, P(opf_mlp_config), vp, ctypes.c_size_t, P(vp)], i32),
        "opf_mlp_destroy": ([vp], i32),
        "opf_mlp_dims": ([vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int64)], i32),
        "opf_mlp_set_params": ([vp, vp, ctypes.c_int64], i32),
        "opf_mlp_get_params": ([vp, vp, ctypes.c_int64], i32),
        "opf_mlp_forward": ([vp, vp, i32, vp], i32),
        "opf_mlp_gradient": ([vp, vp, vp, vp, i32, P(ctypes.c_double), vp], i32),
        "opf_mlp_train": ([vp, vp, vp, vp, i32, i32, i32, ctypes.c_uint64, vp], i32),
        "opf_mlp_pair_gradient": ([vp, vp, vp, i32, vp, i32, P(ctypes.c_double), vp], i32),
        "opf_mlp_train_pairs": ([vp, vp, vp, i32, i32, i32, ctypes.c_uint64, vp], i32),
        "opf_mlp_factors": ([vp, vp, ctypes.c_int64, P(ctypes.c_int32)], i32),
        "opf_precondition": ([vp, vp, vp, vp], i32),
        "opf_mlp_last_error": ([vp], ctypes.c_char_p),
        "opf_ensemble_workspace_size": ([vp, i32, P(ctypes.c_size_t)], i32),
        "opf_ensemble_create": ([vp, i32, vp, ctypes.c_size_t, vp, ctypes.c_char_p, P(vp)], i32),
        "opf_ensemble_tiles": ([vp, P(opf_tiles), i32, P(i32)], i32),
        "opf_autotune": ([vp, i32, ctypes.c_char_p], i32),
        "opf_tile_cache_write": ([P(opf_tiles), i32, ctypes.c_char_p], i32),
        "opf_tile_cache_read": ([ctypes.c_char_p, P(opf_tiles), i32, P(i32)], i32),
        "opf_ensemble_destroy": ([vp], i32),
        "opf_ensemble_member": ([vp, i32, P(vp)], i32),
        "opf_ensemble_step": ([vp, i32], i32),
        "opf_ensemble_tune": ([vp, i32, ctypes.c_char_p, ctypes.c_size_t], i32),
        "opf_ensemble_last_error": ([vp], ctypes.c_char_p),
        "opf_probe_pairs_ensemble": ([vp, vp, dbl, dbl, i32, ctypes.c_uint64, dbl, vp, vp], i32),
        "opf_set_dt": ([vp, dbl], i32),
        "opf_pc_difference": ([vp, P(ctypes.c_double)], i32),
        "opf_step_adaptive": ([vp, i32, P(opf_dt_control), P(ctypes.c_double), P(opf_dt_report)], i32),
        "opf_hookstep_solve": ([P(ctypes.c_double), i32, dbl, dbl, P(ctypes.c_double), P(ctypes.c_double),
                                P(ctypes.c_double)], i32),
        "opf_arnoldi_workspace_size": ([vp, i32, P(ctypes.c_size_t)], i32),
        "opf_arnoldi": ([vp, vp, dbl, dbl, vp, i32, i32, dbl, i32, dbl, vp, ctypes.c_size_t, P(ctypes.c_double),
                         P(ctypes.c_double), P(ctypes.c_double), P(opf_arnoldi_report)], i32),
        "opf_hessenberg_eigvals": ([P(ctypes.c_double), i32, P(ctypes.c_double), P(ctypes.c_double)], i32),
        "opf_set_rotation": ([vp, dbl, dbl, dbl], i32),
        "opf_set_wall_velocity": ([vp, P(ctypes.c_double)], i32),
        "opf_shoot_workspace_size": ([vp, i32, i32, P(ctypes.c_size_t)], i32),
        "opf_shoot_solve": ([vp, vp, P(ctypes.c_double), P(ctypes.c_double), P(opf_shoot_opts), vp, ctypes.c_size_t,
                             P(opf_shoot_report)], i32),
        "opf_status_string": ([i32], ctypes.c_char_p),
        "opf_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def hookstep_solve(Hb, beta, delta):
    """Host-only hookstep subproblem (no device): (y, mu, model residual)."""
    import numpy as np
    lib = load_library()
    Hb = np.ascontiguousarray(Hb, dtype=np.float64)
    k = Hb.shape[1]
    assert Hb.shape == (k + 1, k)
    y = np.zeros(k)
    mu, r = ctypes.c_double(), ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.opf_hookstep_solve(Hb.ctypes.data_as(dp), k, float(beta), float(delta), y.ctypes.data_as(dp),
                                ctypes.byref(mu), ctypes.byref(r))
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())
    return y, mu.value, r.value


def autotune(classes, path):
    """Offline tile tuning of the given classes (keyword dicts for
    make_params), written as a tile cache to `path` (opf_autotune)."""
    lib = load_library()
    n = len(classes)
    params = (opf_params * n)(*[make_params(**c) for c in classes])
    st = lib.opf_autotune(params, n, os.fsencode(path))
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())


def tile_cache_write(entries, path):
    """Write tile-cache entries (dicts with N, M, K, mp, precision, gm, tz,
    ztile) to `path` (host only)."""
    lib = load_library()
    arr = (opf_tiles * len(entries))()
    for i, e in enumerate(entries):
        for k in ("N", "M", "K", "mp", "precision", "gm", "tz", "ztile"):
            setattr(arr[i], k, int(e[k]))
    st = lib.opf_tile_cache_write(arr, len(entries), os.fsencode(path))
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())


def tile_cache_read(path):
    """Entries of a tile cache file, as dicts (host only)."""
    lib = load_library()
    n = ctypes.c_int32()
    st = lib.opf_tile_cache_read(os.fsencode(path), None, 0, ctypes.byref(n))
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())
    arr = (opf_tiles * max(n.value, 1))()
    st = lib.opf_tile_cache_read(os.fsencode(path), arr, n.value, ctypes.byref(n))
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())
    return [arr[i].as_dict() for i in range(n.value)]


def make_params(N=24, M=8, K=8, mp=1, alpha=1.25, Re=2400.0, dt=0.01, c=0.5, n_corr=1,
                fixed_flux=True, precision=OPF_FP64, nonlinear=True, stencil=9):
    p = opf_params()
    p.N, p.M, p.K, p.mp, p.stencil = N, M, K, mp, stencil
    p.alpha, p.Re, p.dt, p.c = alpha, Re, dt, c
    p.n_corr, p.fixed_flux = n_corr, int(bool(fixed_flux))
    p.precision, p.nonlinear = precision, int(bool(nonlinear))
    p.r_nodes = None
    return p


def host_tables(**kw):
    """Create-time radial tables computed on the host (no device needed):
    nodes r, quadrature weights, folded D1 / D2 weights [2][N][9] and the
    stencil start columns."""
    import numpy as np
    lib = load_library()
    p = make_params(**kw)
    N = p.N
    r, q = np.zeros(N), np.zeros(N)
    d1, d2 = np.zeros((2, N, 9)), np.zeros((2, N, 9))
    s0 = np.zeros(N, dtype=np.int32)
    st = lib.opf_tables(ctypes.byref(p), r.ctypes.data, q.ctypes.data, d1.ctypes.data,
                        d2.ctypes.data, s0.ctypes.data)
    if st != OPF_OK:
        raise OpfError(st, lib.opf_status_string(st).decode())
    return r, q, d1, d2, s0


class Solver:
    """One time-step context on the current CUDA/HIP device.

    State tensors are complex128 of shape [3][M][2K-1][N] on the device.
    """

    def __init__(self, r_nodes=None, stream=None, **kw):
        import numpy as np
        import torch
        self.torch = torch
        self.lib = load_library()
        self.kw = dict(kw)
        self.p = make_params(**kw)
        self._nodes = None
        if r_nodes is not None:
            self._nodes = np.ascontiguousarray(r_nodes, dtype=np.float64)
            self.p.r_nodes = self._nodes.ctypes.data
        nbytes = ctypes.c_size_t()
        self._check(self.lib.opf_workspace_size(ctypes.byref(self.p), ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        self._check(self.lib.opf_create(ctypes.byref(self.p), ctypes.c_void_p(self._ws_ptr),
                                        ctypes.c_size_t(self.ws_bytes),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self.N, self.M, self.K = self.p.N, self.p.M, self.p.K
        self.shape = (3, self.M, 2 * self.K - 1, self.N)

    def _check(self, st, ctx=None):
        if st != OPF_OK:
            msg = self.lib.opf_status_string(st).decode()
            c = ctx if ctx is not None else getattr(self, "ctx", None)
            if c is not None:
                detail = self.lib.opf_last_error(c)
                if detail:
                    msg += ": " + detail.decode()
            raise OpfError(st, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.opf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------
    def _dev(self, t, shape=None, dtype=None):
        torch = self.torch
        t = torch.as_tensor(t)
        if dtype is None:
            dtype = torch.complex128
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise OpfError(OPF_E_INVALID, f"expected shape {shape}, got {tuple(t.shape)}")
        return t

    def nodes(self):
        import numpy as np
        r = np.zeros(self.N)
        self._check(self.lib.opf_get_nodes(self.ctx, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return r

    # -- ABI calls ------------------------------------------------------
    def set_state(self, u):
        u = self._dev(u, self.shape)
        self._check(self.lib.opf_set_state(self.ctx, ctypes.c_void_p(u.data_ptr())))
        self.stream.synchronize()

    def get_state(self):
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        self._check(self.lib.opf_get_state(self.ctx, ctypes.c_void_p(out.data_ptr())))
        return out

    def step(self, n=1):
        self._check(self.lib.opf_step(self.ctx, int(n)))

    def set_wall_velocity(self, b):
        """Prescribed wall velocity b [3, M, 2K-1] complex (r, theta, z at
        r = 1) through the influence-matrix vector g; None restores no slip."""
        import numpy as np
        if b is None:
            self._check(self.lib.opf_set_wall_velocity(self.ctx, None))
            return
        b = np.ascontiguousarray(b, dtype=np.complex128)
        if b.shape != tuple(self.shape[:3]):
            raise OpfError(OPF_E_INVALID, f"expected shape {tuple(self.shape[:3])}, got {b.shape}")
        self._check(self.lib.opf_set_wall_velocity(self.ctx, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def set_rotation(self, ox, oy, oz):
        """Coriolis force -2 Omega x u on the nonlinear term (Omega Cartesian,
        z the pipe axis, units U_cl / R; all zero switches it off)."""
        self._check(self.lib.opf_set_rotation(self.ctx, float(ox), float(oy), float(oz)))

    def set_dt(self, dt):
        """Rebuild the dt-dependent operator tables for a new step size."""
        self._check(self.lib.opf_set_dt(self.ctx, float(dt)))
        self.p.dt = float(dt)

    def pc_difference(self):
        """||u^{n+1} - u^p|| (energy norm) of the last step."""
        out = ctypes.c_double()
        self._check(self.lib.opf_pc_difference(self.ctx, ctypes.byref(out)))
        return out.value

    def step_adaptive(self, n, courant=0.5, pc_tol=0.0, dt_min=1e-6, dt_max=0.05, grow=0.1, check_every=10,
                      trace=False):
        """n steps under automatic time-step control; returns the report as a
        dict (with "dts", the step size of every step, when trace=True)."""
        ctl = opf_dt_control(float(courant), float(pc_tol), float(dt_min), float(dt_max), float(grow),
                             int(check_every))
        rep = opf_dt_report()
        buf = (ctypes.c_double * max(int(n), 1))() if trace else None
        st = self.lib.opf_step_adaptive(self.ctx, int(n), ctypes.byref(ctl), buf, ctypes.byref(rep))
        self.p.dt = rep.dt
        self._check(st)
        out = {name: getattr(rep, name) for name, _ in opf_dt_report._fields_}
        if trace:
            out["dts"] = list(buf)[:int(n)]
        return out

    def nonlinear(self, u):
        u = self._dev(u, self.shape)
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        self._check(self.lib.opf_nonlinear(self.ctx, ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr())))
        return out

    def vorticity(self, u):
        u = self._dev(u, self.shape)
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        self._check(self.lib.opf_vorticity(self.ctx, ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr())))
        return out

    def radial_solve(self, kind, rhs, want_pressure=False):
        nf = 6 if kind == OPF_SOLVE_CORR else 3
        rhs = self._dev(rhs, (nf,) + self.shape[1:])
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        p = None
        if want_pressure:
            p = self.torch.zeros(self.shape[1:], dtype=self.torch.complex128, device=self.device)
        self._check(self.lib.opf_radial_solve(
            self.ctx, int(kind), ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(p.data_ptr() if p is not None else 0)))
        return (out, p) if want_pressure else out

    def newton_residual(self, x, T, shift):
        x = self._dev(x, self.shape)
        F = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        nrm = ctypes.c_double()
        self._check(self.lib.opf_newton_residual(self.ctx, ctypes.c_void_p(x.data_ptr()), float(T),
                                                 float(shift), ctypes.c_void_p(F.data_ptr()),
                                                 ctypes.byref(nrm)))
        return F, nrm.value

    KERNELS = ("zinv", "theta", "zfwd", "solve_pred", "solve_corr")

    def profile_steps(self, n):
        """Per-kernel device time (ms, summed) and launch counts over n
        eagerly launched steps, from HIP events on the context's stream."""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int32 * 5)()
        self._check(self.lib.opf_profile_steps(self.ctx, int(n), ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def vec_dot(self, a, b):
        a, b = self._dev(a, self.shape), self._dev(b, self.shape)
        out = ctypes.c_double()
        self._check(self.lib.opf_vec_dot(self.ctx, ctypes.c_void_p(a.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), ctypes.byref(out)))
        return out.value

    def nk_solve(self, x, T, speed=0.0, free_speed=False, gmres_m=40, max_newton=20, max_jvps=400, tol=1e-8,
                 gmres_tol=1e-3, fd_eps=1e-7, precond=None, record=None, hookstep=False, tr_delta0=0.0,
                 tr_delta_max=0.0, max_hook=12, fallback=True, speed_freeze=0.0):
        """Newton-Krylov travelling-wave search; returns (solution, report dict).
        speed: the phase speed c_w (shift c_w T), solved for when free_speed.
        precond: an Mlp (flexible GMRES with it as right preconditioner) or None;
        plain GMRES is its fallback unless fallback=False.
        record: None, or a complex128 device tensor [n, 2, 3, M, 2K-1, N] that
        receives the pairs (z, J z) of the products the solver forms.
        hookstep: the Krylov trust-region step instead of restarted GMRES and
        a line search (tr_delta0 <= 0: first radius = first Newton step)."""
        x = self._dev(x, self.shape).clone()
        nbytes = ctypes.c_size_t()
        self._check(self.lib.opf_nk_workspace_size(self.ctx, int(gmres_m), int(precond is not None),
                                                    ctypes.byref(nbytes)))
        kry = self.torch.empty(nbytes.value, dtype=self.torch.uint8, device=self.device)
        cap = 0
        if record is not None:
            assert record.is_cuda and record.dtype == self.torch.complex128 and record.is_contiguous()
            assert tuple(record.shape[1:]) == (2,) + tuple(self.shape)
            cap = record.shape[0]
        o = opf_nk_opts(int(gmres_m), int(max_newton), int(max_jvps), float(tol), float(gmres_tol),
                        float(fd_eps), precond.handle if precond is not None else None,
                        record.data_ptr() if record is not None else None, int(cap), int(bool(hookstep)),
                        float(tr_delta0), float(tr_delta_max), int(max_hook), int(bool(free_speed)),
                        int(not fallback), float(speed_freeze))
        rep = opf_nk_report()
        cw = ctypes.c_double(float(speed))
        self._check(self.lib.opf_nk_solve(self.ctx, ctypes.c_void_p(x.data_ptr()), float(T), ctypes.byref(cw),
                                          ctypes.byref(o), ctypes.c_void_p(kry.data_ptr()),
                                          ctypes.c_size_t(nbytes.value), ctypes.byref(rep)))
        n = rep.newton_iterations
        return x, {"newton_iterations": n, "gmres_iterations": rep.gmres_iterations,
                   "jvps": rep.jvps, "converged": bool(rep.converged), "residual": rep.residual,
                   "history": [rep.residual_history[i] for i in range(min(n + 1, 32))],
                   "recorded": rep.recorded, "precond_applies": rep.precond_applies,
                   "residual_evals": rep.residual_evals, "hook_trials": rep.hook_trials,
                   "stalled": bool(rep.stalled), "tr_delta": rep.tr_delta, "speed": cw.value,
                   "frozen_steps": rep.frozen_steps, "fallbacks": rep.fallbacks}

    def shoot_solve(self, xs, T, shift, steps, free_T=True, free_s=True, gmres_m=40, max_newton=20, tol=1e-8,
                    gmres_tol=1e-3, fd_eps=1e-7, tr_delta0=0.0, tr_delta_max=0.0, max_hook=12):
        """Relative periodic orbit by multiple shooting: xs [S, 3, M, 2K-1, N]
        section states, period T, shift s, `steps` steps per section.
        Returns (sections, T, s, report dict)."""
        xs = self._dev(xs, tuple(xs.shape[:1]) + tuple(self.shape)).clone()
        S = xs.shape[0]
        nbytes = ctypes.c_size_t()
        self._check(self.lib.opf_shoot_workspace_size(self.ctx, int(S), int(gmres_m), ctypes.byref(nbytes)))
        work = self.torch.empty(nbytes.value, dtype=self.torch.uint8, device=self.device)
        o = opf_shoot_opts(int(S), int(steps), int(bool(free_T)), int(bool(free_s)), int(gmres_m), int(max_newton),
                           float(tol), float(gmres_tol), float(fd_eps), float(tr_delta0), float(tr_delta_max),
                           int(max_hook))
        Tc, sc = ctypes.c_double(T), ctypes.c_double(shift)
        rep = opf_shoot_report()
        self._check(self.lib.opf_shoot_solve(self.ctx, ctypes.c_void_p(xs.data_ptr()), ctypes.byref(Tc),
                                             ctypes.byref(sc), ctypes.byref(o), ctypes.c_void_p(work.data_ptr()),
                                             ctypes.c_size_t(nbytes.value), ctypes.byref(rep)))
        n = rep.newton_iterations
        return xs, Tc.value, sc.value, {
            "newton_iterations": n, "products": rep.products, "residual_evals": rep.residual_evals,
            "hook_trials": rep.hook_trials, "converged": bool(rep.converged), "stalled": bool(rep.stalled),
            "residual": rep.residual, "history": [rep.residual_history[i] for i in range(min(n + 1, 32))],
            "tr_delta": rep.tr_delta}

    def arnoldi(self, x, T, shift, v0, m=40, nev=6, tol=1e-8, check_every=5, fd_eps=1e-7):
        """Leading Floquet multipliers of the time-T map at x (shifted by
        -shift): (complex numpy array of nev Ritz values, report dict with
        the Hessenberg matrix)."""
        import numpy as np
        x = self._dev(x, self.shape)
        v0 = self._dev(v0, self.shape)
        nbytes = ctypes.c_size_t()
        self._check(self.lib.opf_arnoldi_workspace_size(self.ctx, int(m), ctypes.byref(nbytes)))
        work = self.torch.empty(nbytes.value, dtype=self.torch.uint8, device=self.device)
        re, im = np.zeros(int(nev)), np.zeros(int(nev))
        hess = np.zeros((int(m) + 1, int(m)))
        rep = opf_arnoldi_report()
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.opf_arnoldi(self.ctx, ctypes.c_void_p(x.data_ptr()), float(T), float(shift),
                                         ctypes.c_void_p(v0.data_ptr()), int(m), int(nev), float(tol),
                                         int(check_every), float(fd_eps), ctypes.c_void_p(work.data_ptr()),
                                         ctypes.c_size_t(nbytes.value), re.ctypes.data_as(dp), im.ctypes.data_as(dp),
                                         hess.ctypes.data_as(dp), ctypes.byref(rep)))
        k = rep.products
        return re + 1j * im, {"products": k, "converged": bool(rep.converged), "checks": rep.checks,
                              "hessenberg": hess[:k + 1, :k]}

    def probe_pairs(self, x, T, shift, n, seed=1, fd_eps=1e-7, batch=1):
        """n Jacobian probes (z, J z) of the travelling-wave residual at x:
        complex128 device tensor [n, 2, 3, M, 2K-1, N].  batch > 1 runs the
        probes' trajectories `batch` at a time as ensemble members (same
        pairs, bitwise)."""
        x = self._dev(x, self.shape)
        pairs = self.torch.empty((int(n), 2) + tuple(self.shape), dtype=self.torch.complex128, device=self.device)
        work = self.torch.empty((3,) + tuple(self.shape), dtype=self.torch.complex128, device=self.device)
        args = (ctypes.c_void_p(x.data_ptr()), float(T), float(shift), int(n), int(seed), float(fd_eps),
                ctypes.c_void_p(pairs.data_ptr()), ctypes.c_void_p(work.data_ptr()))
        if batch > 1:
            kw = dict(self.kw)
            if self._nodes is not None:
                kw["r_nodes"] = self._nodes
            ens = Ensemble([kw] * int(batch), stream=self.stream)
            try:
                ens._check(self.lib.opf_probe_pairs_ensemble(ens.ens, *args))
            finally:
                ens.close()
        else:
            self._check(self.lib.opf_probe_pairs(self.ctx, *args))
        return pairs

    def probe_pairs_noalloc(self, x, T, shift, n, seed=1, fd_eps=1e-7):
        """opf_probe_pairs_noalloc: the pairs of probe_pairs, with the
        library's static device scratch as work space (no workspace
        argument; see opf.h)."""
        x = self._dev(x, self.shape)
        pairs = self.torch.empty((int(n), 2) + tuple(self.shape), dtype=self.torch.complex128, device=self.device)
        self._check(self.lib.opf_probe_pairs_noalloc(self.ctx, ctypes.c_void_p(x.data_ptr()), float(T),
                                                     float(shift), int(n), int(seed), float(fd_eps),
                                                     ctypes.c_void_p(pairs.data_ptr())))
        return pairs

    def diagnostics(self, check=True):
        """Diagnostics dict; with check=False a non-finite value or CFL > 1
        is reported in the dict ("status") instead of raising."""
        d = opf_diag()
        st = self.lib.opf_diagnostics(self.ctx, ctypes.byref(d))
        if check:
            self._check(st)
        out = {name: getattr(d, name) for name, _ in opf_diag._fields_}
        out["status"] = st
        return out


class _Member(Solver):
    """A member context of an Ensemble (owned by the ensemble)."""

    def __init__(self, ens, i, params):
        import torch
        self.torch = torch
        self.lib = ens.lib
        self.p = params
        self.device = ens.device
        self.stream = ens.stream
        ctx = ctypes.c_void_p()
        ens._check(self.lib.opf_ensemble_member(ens.ens, i, ctypes.byref(ctx)))
        self.ctx = ctx
        self.N, self.M, self.K = params.N, params.M, params.K
        self.shape = (3, self.M, 2 * self.K - 1, self.N)

    def close(self):  # owned by the ensemble
        self.ctx = None


class Ensemble:
    """Independent trajectories stepped together (one graph launch per step).
    `members` is a list of keyword dicts for make_params."""

    def __init__(self, members, stream=None, tune_cache=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        import numpy as np
        n = len(members)
        self._nodes = []  # explicit radial nodes of members that give them (kept alive)
        plist = []
        for m in members:
            m = dict(m)
            r = m.pop("r_nodes", None)
            p = make_params(**m)
            if r is not None:
                r = np.ascontiguousarray(r, dtype=np.float64)
                self._nodes.append(r)
                p.r_nodes = r.ctypes.data
            plist.append(p)
        self.params = (opf_params * n)(*plist)
        nbytes = ctypes.c_size_t()
        self.ens = None
        self._check(self.lib.opf_ensemble_workspace_size(self.params, n, ctypes.byref(nbytes)))
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ens = ctypes.c_void_p()
        self._check(self.lib.opf_ensemble_create(self.params, n, ctypes.c_void_p(ptr), nbytes.value,
                                                 ctypes.c_void_p(self.stream.cuda_stream),
                                                 None if tune_cache is None else os.fsencode(tune_cache),
                                                 ctypes.byref(ens)))
        self.ens = ens
        self.members = [_Member(self, i, self.params[i]) for i in range(n)]

    def _check(self, st):
        if st != OPF_OK:
            msg = self.lib.opf_status_string(st).decode()
            if getattr(self, "ens", None):
                msg += ": " + self.lib.opf_ensemble_last_error(self.ens).decode()
            raise OpfError(st, msg)

    def step(self, n=1):
        self._check(self.lib.opf_ensemble_step(self.ens, int(n)))

    def tune(self, nsteps=5):
        """Tile autotuning (see opf_ensemble_tune); returns the tile cache as
        a dict (json.dump it to a file for Ensemble(tune_cache=...))."""
        import json
        buf = ctypes.create_string_buffer(1 << 18)
        self._check(self.lib.opf_ensemble_tune(self.ens, int(nsteps), buf, len(buf)))
        return json.loads(buf.value.decode())

    def tiles(self):
        """Current tile shapes per class, as dicts."""
        n = ctypes.c_int32()
        self._check(self.lib.opf_ensemble_tiles(self.ens, None, 0, ctypes.byref(n)))
        out = (opf_tiles * max(n.value, 1))()
        self._check(self.lib.opf_ensemble_tiles(self.ens, out, n.value, ctypes.byref(n)))
        return [out[i].as_dict() for i in range(n.value)]

    def close(self):
        if getattr(self, "ens", None):
            self.lib.opf_ensemble_destroy(self.ens)
            self.ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Learned preconditioner of a Solver's grid (see opf.h): a residual MLP
    on the matrix cores turns each mode's features into the factors of a
    rank-R correction of -I; trained with Adam on recorded (z, J z) pairs and
    applied by Solver.nk_solve(precond=...)."""

    def __init__(self, solver, width=256, layers=4, rank=8, max_rows=0, seed=1, lr=1e-3, beta1=0.9,
                 beta2=0.999, adam_eps=1e-8, lr_final=None):
        import torch
        self.torch = torch
        self.solver = solver  # the context must outlive the network
        self.lib = solver.lib
        self.mode_rows = solver.M * (2 * solver.K - 1)
        cfg = opf_mlp_config()
        solver._check(self.lib.opf_mlp_default_config(ctypes.byref(cfg)))
        cfg.width, cfg.layers, cfg.rank, cfg.seed = int(width), int(layers), int(rank), int(seed)
        cfg.max_rows = int(max_rows)
        cfg.lr, cfg.beta1, cfg.beta2, cfg.adam_eps = lr, beta1, beta2, adam_eps
        cfg.lr_final = lr if lr_final is None else lr_final
        self.cfg = cfg
        self.layers, self.rank, self.width = int(layers), int(rank), int(width)
        nbytes = ctypes.c_size_t()
        solver._check(self.lib.opf_mlp_workspace_size(solver.ctx, ctypes.byref(cfg), ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=solver.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        solver._check(self.lib.opf_mlp_create(solver.ctx, ctypes.byref(cfg), ctypes.c_void_p(ptr),
                                              ctypes.c_size_t(nbytes.value), ctypes.byref(h)))
        self.handle = h.value
        din, dout, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.opf_mlp_dims(self.handle, ctypes.byref(din), ctypes.byref(dout), ctypes.byref(n)))
        self.din, self.dout, self.n_params = din.value, dout.value, n.value

    def _check(self, st):
        if st != OPF_OK:
            msg = self.lib.opf_status_string(st).decode()
            if getattr(self, "handle", None):
                detail = self.lib.opf_mlp_last_error(self.handle)
                if detail:
                    msg += ": " + detail.decode()
            raise OpfError(st, msg)

    def _rows(self, t, width):
        t = self.torch.as_tensor(t).to(device=self.solver.device, dtype=self.torch.float32).contiguous()
        if t.dim() != 2 or t.shape[1] != width:
            raise OpfError(OPF_E_INVALID, f"expected rows of width {width}, got {tuple(t.shape)}")
        return t

    def _pairs(self, pairs):
        s = self.solver
        pairs = s._dev(pairs).contiguous()
        if tuple(pairs.shape[1:]) != (2,) + tuple(s.shape):
            raise OpfError(OPF_E_INVALID, f"pairs must be [n, 2, {s.shape}], got {tuple(pairs.shape)}")
        return pairs

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(self.lib.opf_mlp_set_params(self.handle, ctypes.c_void_p(a.ctypes.data), a.size))

    def get_params(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.opf_mlp_get_params(self.handle, ctypes.c_void_p(a.ctypes.data), a.size))
        return a

    def forward(self, x):
        x = self._rows(x, self.din)
        y = self.torch.empty((x.shape[0], self.dout), dtype=self.torch.float32, device=x.device)
        self._check(self.lib.opf_mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                             ctypes.c_void_p(y.data_ptr())))
        return y

    def gradient(self, x, t, w=None):
        import numpy as np
        x, t = self._rows(x, self.din), self._rows(t, self.dout)
        wp = None
        if w is not None:
            w = self.torch.as_tensor(w).to(device=x.device, dtype=self.torch.float32).contiguous()
            wp = w.data_ptr()
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self.lib.opf_mlp_gradient(self.handle, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(wp), x.shape[0],
                                              ctypes.byref(loss), ctypes.c_void_p(g.ctypes.data)))
        return loss.value, g

    def train(self, x, t, w=None, batch=None, epochs=1, seed=1):
        import numpy as np
        x, t = self._rows(x, self.din), self._rows(t, self.dout)
        wp = None
        if w is not None:
            w = self.torch.as_tensor(w).to(device=x.device, dtype=self.torch.float32).contiguous()
            wp = w.data_ptr()
        batch = int(batch if batch is not None else x.shape[0])
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        self._check(self.lib.opf_mlp_train(self.handle, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(wp), x.shape[0],
                                           batch, int(epochs), int(seed), ctypes.c_void_p(losses.ctypes.data)))
        return losses[:epochs]

    def pair_gradient(self, pairs, idx):
        """Pair loss of pairs[idx] and its parameter gradient (no update)."""
        import numpy as np
        s = self.solver
        pairs = self._pairs(pairs)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        s._check(self.lib.opf_mlp_pair_gradient(s.ctx, self.handle, ctypes.c_void_p(pairs.data_ptr()),
                                                pairs.shape[0], ctypes.c_void_p(idx.ctypes.data), idx.size,
                                                ctypes.byref(loss), ctypes.c_void_p(g.ctypes.data)))
        return loss.value, g

    def train_pairs(self, pairs, batch=16, steps=1000, seed=1):
        """Adam on recorded (z, J z) pairs [n, 2, 3, M, 2K-1, N]; returns the
        per-step losses."""
        import numpy as np
        s = self.solver
        pairs = self._pairs(pairs)
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        s._check(self.lib.opf_mlp_train_pairs(s.ctx, self.handle, ctypes.c_void_p(pairs.data_ptr()),
                                              pairs.shape[0], int(batch), int(steps), int(seed),
                                              ctypes.c_void_p(losses.ctypes.data)))
        return losses[:steps]

    def factors(self):
        """Preconditioner factor rows (A, B) and the count of modes left at -I."""
        import numpy as np
        f = np.zeros((self.mode_rows, self.dout), dtype=np.float32)
        bad = ctypes.c_int32()
        self._check(self.lib.opf_mlp_factors(self.handle, ctypes.c_void_p(f.ctypes.data), f.size,
                                             ctypes.byref(bad)))
        return f, bad.value

    def precondition(self, v):
        s = self.solver
        v = s._dev(v, s.shape)
        z = self.torch.empty_like(v)
        s._check(self.lib.opf_precondition(s.ctx, self.handle, ctypes.c_void_p(v.data_ptr()),
                                           ctypes.c_void_p(z.data_ptr())))
        return z

    def close(self):
        if getattr(self, "handle", None):
            self.lib.opf_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
