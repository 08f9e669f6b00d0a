"""ctypes binding of libstp.so (include/stp.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory and the stream.  The module-level functions
carry the C names; ``SpaceTimeSolver`` wraps one context.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libstp.so")
_lib = None

STP_OK, STP_EINVAL, STP_ENOMEM, STP_EDEVICE, STP_ENOTCONV, STP_EDIVERGED, STP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STP_PREC = {"f64": 0, "f32": 1, "bf16": 2}
STP_SPATIAL = {"auto": 0, "mg": 1, "exact": 2, "none": 3}
STP_OP_B, STP_OP_SADDLE = 0, 1
STP_PC_A, STP_PC_H = 0, 1
STP_MAX_RANK = 4


class StpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class stp_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int)]


class stp_kappa(C.Structure):
    _fields_ = [("rank", C.c_int), ("fields", C.c_void_p), ("tcoef", C.POINTER(C.c_double))]


class stp_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("spatial", C.c_int), ("nu_A", C.c_int), ("nu_H", C.c_int),
                ("omega", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int),
                ("kref_coef", C.POINTER(C.c_double)), ("check_every", C.c_int), ("use_graph", C.c_int),
                ("tau_steps", C.POINTER(C.c_double)), ("disc", C.c_int),
                ("sweeps", C.c_int)]


STP_NPHASE = 5
PHASES = ("resid", "atilde", "dst", "hblock", "other")   # STP_PHASE_* order


class stp_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res", C.c_double), ("omega_used", C.c_double),
                ("t_solve_ms", C.c_double), ("status", C.c_int), ("rel_rp", C.c_double),
                ("rel_ru", C.c_double), ("t_setup_ms", C.c_double), ("t_omega_ms", C.c_double),
                ("t_phase_ms", C.c_double * STP_NPHASE)]


def stats_dict(st, status=None):
    """The fields of an stp_stats as a dict (status: the call's return code if given)."""
    return dict(status=st.status if status is None else status, iters=st.iters, rel_res=st.rel_res,
                omega=st.omega_used, ms=st.t_solve_ms, rel_rp=st.rel_rp, rel_ru=st.rel_ru,
                setup_ms=st.t_setup_ms, omega_ms=st.t_omega_ms,
                phase_ms=dict(zip(PHASES, list(st.t_phase_ms))))


class stp_tune_report(C.Structure):
    _fields_ = [("knobs_tuned", C.c_int), ("candidates", C.c_int), ("from_cache", C.c_int),
                ("iter_ms_before", C.c_double), ("iter_ms_after", C.c_double)]


def lib_path() -> str:
    return _LIB_PATH


def load() -> C.CDLL:
    """Load libstp.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libstp.so not built at {_LIB_PATH}; run python -m paper_1802_08126_amd.build_lib")
    lib = C.CDLL(_LIB_PATH)
    lib.stp_default_options.argtypes = [C.POINTER(stp_options)]
    lib.stp_default_options.restype = None
    lib.stp_workspace_bytes.argtypes = [C.POINTER(stp_grid), C.c_int, C.c_int, C.POINTER(stp_options)]
    lib.stp_workspace_bytes.restype = C.c_size_t
    lib.stp_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(stp_grid), C.c_int, C.c_double,
                               C.POINTER(stp_kappa), C.c_void_p, C.c_void_p, C.POINTER(stp_options),
                               C.c_void_p, C.c_size_t, C.c_void_p]
    lib.stp_create.restype = C.c_int
    lib.stp_apply_operator.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    lib.stp_apply_operator.restype = C.c_int
    lib.stp_apply_precond.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    lib.stp_apply_precond.restype = C.c_int
    lib.stp_uzawa_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(stp_stats)]
    lib.stp_uzawa_solve.restype = C.c_int
    lib.stp_destroy.argtypes = [C.c_void_p]
    lib.stp_destroy.restype = None
    lib.stp_status_string.argtypes = [C.c_int]
    lib.stp_status_string.restype = C.c_char_p
    lib.stp_last_error.argtypes = []
    lib.stp_last_error.restype = C.c_char_p
    lib.stp_workspace_bytes_batch.argtypes = [C.c_int, C.POINTER(stp_grid), C.POINTER(C.c_int),
                                              C.POINTER(C.c_int), C.POINTER(stp_options)]
    lib.stp_workspace_bytes_batch.restype = C.c_size_t
    lib.stp_create_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(stp_grid), C.POINTER(C.c_int),
                                     C.POINTER(C.c_double), C.POINTER(stp_kappa), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(stp_options), C.c_void_p, C.c_size_t,
                                     C.c_void_p]
    lib.stp_create_batch.restype = C.c_int
    lib.stp_uzawa_solve_batch.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.POINTER(stp_stats)]
    lib.stp_uzawa_solve_batch.restype = C.c_int
    lib.stp_batch_size.argtypes = [C.c_void_p]
    lib.stp_batch_size.restype = C.c_int
    lib.stp_device_bytes_allocated.argtypes = []
    lib.stp_device_bytes_allocated.restype = C.c_size_t
    lib.stp_set_stop.argtypes = [C.c_void_p, C.c_double, C.c_int]
    lib.stp_set_stop.restype = C.c_int
    lib.stp_gmres_solve_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                            C.POINTER(C.c_double), C.POINTER(stp_stats)]
    lib.stp_gmres_solve_noalloc.restype = C.c_int
    lib.stp_omega_info.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
    lib.stp_omega_info.restype = C.c_int
    lib.stp_set_omega.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
    lib.stp_set_omega.restype = C.c_int
    lib.stp_gmres_workspace_bytes.argtypes = [C.c_void_p, C.c_int]
    lib.stp_gmres_workspace_bytes.restype = C.c_size_t
    lib.stp_gmres_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t,
                                    C.POINTER(C.c_double), C.POINTER(stp_stats)]
    lib.stp_gmres_solve.restype = C.c_int
    lib.stp_autotune.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(stp_tune_report)]
    lib.stp_autotune.restype = C.c_int
    lib.stp_schedule_string.argtypes = [C.c_void_p]
    lib.stp_schedule_string.restype = C.c_char_p
    lib.stp_timing_enable.argtypes = [C.c_void_p, C.c_int]
    lib.stp_timing_enable.restype = C.c_int
    lib.stp_timing_count.argtypes = [C.c_void_p]
    lib.stp_timing_count.restype = C.c_int
    lib.stp_timing_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_int),
                                   C.POINTER(C.c_long), C.POINTER(C.c_double)]
    lib.stp_timing_get.restype = C.c_int
    _lib = lib
    return lib


def _check(status, what):
    if status != STP_OK:
        lib = load()
        raise StpError(status, f"{what}: {lib.stp_status_string(status).decode()}: {lib.stp_last_error().decode()}")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape) and t.numel() != int(np.prod(shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


STP_DISC = {"fd": 0, "fem": 1}


def make_options(precision="f64", spatial="auto", omega=0.8, tol=1e-8, max_iter=500, kref_coef=None,
                 check_every=8, use_graph=True, nu_A=1, nu_H=1, tau_steps=None, disc="fd", sweeps=1):
    o = stp_options()
    load().stp_default_options(C.byref(o))
    o.disc = STP_DISC[disc]
    o.sweeps = sweeps
    o.precision = STP_PREC[precision]
    o.spatial = STP_SPATIAL[spatial]
    o.nu_A, o.nu_H = nu_A, nu_H
    o.omega = omega
    o.tol = tol
    o.max_iter = max_iter
    o.check_every = check_every
    o.use_graph = 1 if use_graph else 0
    keep = []
    if kref_coef is not None:
        keep.append((C.c_double * len(kref_coef))(*[float(v) for v in kref_coef]))
        o.kref_coef = C.cast(keep[-1], C.POINTER(C.c_double))
    if tau_steps is not None:
        keep.append((C.c_double * len(tau_steps))(*[float(v) for v in tau_steps]))
        o.tau_steps = C.cast(keep[-1], C.POINTER(C.c_double))
    return o, keep


# --- C-named entry points ------------------------------------------------------

def stp_workspace_bytes(dim, n, N, rank, **opts) -> int:
    o, _keep = make_options(**opts)
    g = stp_grid(dim, n)
    return int(load().stp_workspace_bytes(C.byref(g), N, rank, C.byref(o)))


def stp_create(dim, n, N, tau, kfields, tcoef, F, u0, workspace=None, stream=None, **opts):
    """Returns (ctx handle, keepalive tuple).  kfields, F, u0 are CUDA float64 tensors
    (borrowed: keep them alive until stp_destroy); tcoef is host (rank x N)."""
    lib = load()
    tcoef = np.ascontiguousarray(np.asarray(tcoef, dtype=np.float64))
    R = tcoef.shape[0]
    if tcoef.shape != (R, N) or not (1 <= R <= STP_MAX_RANK):
        raise ValueError(f"tcoef must be (rank, N) with rank <= {STP_MAX_RANK}, got {tcoef.shape}")
    npts = n ** dim
    kf = _dev_f64(kfields, (R,) + (n + 2,) * dim, "kfields")
    Fp = _dev_f64(F, (N,) + (n,) * dim, "F")
    up = _dev_f64(u0, (n,) * dim, "u0")
    if kfields.numel() != R * (n + 2) ** dim or F.numel() != N * npts or u0.numel() != npts:
        raise ValueError("kfields/F/u0 sizes do not match (dim, n, N, rank)")
    if opts.get("tau_steps") is not None and len(opts["tau_steps"]) != N:
        raise ValueError(f"tau_steps must hold N = {N} step lengths, got {len(opts['tau_steps'])}")
    o, keep = make_options(**opts)
    g = stp_grid(dim, n)
    tc = tcoef.ctypes.data_as(C.POINTER(C.c_double))
    kap = stp_kappa(R, kf, tc)
    ctx = C.c_void_p()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    st = lib.stp_create(C.byref(ctx), C.byref(g), N, float(tau), C.byref(kap), Fp, up, C.byref(o),
                        ws_ptr, ws_bytes, _stream_ptr(stream))
    _check(st, "stp_create")
    return ctx, (kfields, F, u0, tcoef, keep, workspace)


def stp_workspace_bytes_batch(specs, **opts) -> int:
    """specs: list of (dim, n, N, rank)."""
    P = len(specs)
    o, _keep = make_options(**opts)
    grids = (stp_grid * P)(*[stp_grid(d, n) for d, n, _, _ in specs])
    Ns = (C.c_int * P)(*[N for _, _, N, _ in specs])
    rk = (C.c_int * P)(*[r for _, _, _, r in specs])
    return int(load().stp_workspace_bytes_batch(P, grids, Ns, rk, C.byref(o)))


def stp_create_batch(problems, workspace=None, stream=None, **opts):
    """problems: list of dicts with keys dim, n, N, tau, kfields, tcoef, F, u0 (as in
    stp_create) and optionally steps (N step lengths; tau is then the reference
    step).  Without a tau_steps option the steps of the problems that give them
    (N copies of tau for the others) form it.  Returns (ctx handle, keepalive tuple)."""
    lib = load()
    P = len(problems)
    if P < 1:
        raise ValueError("empty batch")
    grids = (stp_grid * P)()
    Ns = (C.c_int * P)()
    taus = (C.c_double * P)()
    kaps = (stp_kappa * P)()
    Fs = (C.c_void_p * P)()
    u0s = (C.c_void_p * P)()
    keep = []
    for i, q in enumerate(problems):
        dim, n, N = q["dim"], q["n"], q["N"]
        tcoef = np.ascontiguousarray(np.asarray(q["tcoef"], dtype=np.float64))
        R = tcoef.shape[0]
        if tcoef.shape != (R, N) or not (1 <= R <= STP_MAX_RANK):
            raise ValueError(f"problem {i}: tcoef must be (rank, N) with rank <= {STP_MAX_RANK}, got {tcoef.shape}")
        npts = n ** dim
        kf, F, u0 = q["kfields"], q["F"], q["u0"]
        if kf.numel() != R * (n + 2) ** dim or F.numel() != N * npts or u0.numel() != npts:
            raise ValueError(f"problem {i}: kfields/F/u0 sizes do not match (dim, n, N, rank)")
        grids[i] = stp_grid(dim, n)
        Ns[i] = N
        taus[i] = float(q["tau"])
        kaps[i] = stp_kappa(R, _dev_f64(kf, (R,) + (n + 2,) * dim, "kfields"),
                            tcoef.ctypes.data_as(C.POINTER(C.c_double)))
        Fs[i] = _dev_f64(F, (N,) + (n,) * dim, "F").value
        u0s[i] = _dev_f64(u0, (n,) * dim, "u0").value
        keep.append((kf, F, u0, tcoef))
    total = sum(q["N"] for q in problems)
    if opts.get("tau_steps") is None and any(q.get("steps") is not None for q in problems):
        opts["tau_steps"] = [float(v) for q in problems
                             for v in (q["steps"] if q.get("steps") is not None else [q["tau"]] * q["N"])]
    if opts.get("tau_steps") is not None and len(opts["tau_steps"]) != total:
        raise ValueError(f"tau_steps must hold sum(N) = {total} step lengths, got {len(opts['tau_steps'])}")
    o, okeep = make_options(**opts)
    ctx = C.c_void_p()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    st = lib.stp_create_batch(C.byref(ctx), P, grids, Ns, taus, kaps, Fs, u0s, C.byref(o), ws_ptr, ws_bytes,
                              _stream_ptr(stream))
    _check(st, "stp_create_batch")
    return ctx, (keep, okeep, workspace)


def stp_uzawa_solve_batch(ctx, us, ps):
    """Returns (worst status, list of stp_stats)."""
    P = len(us)
    if len(ps) != P:
        raise ValueError("u and p lists differ in length")
    ua = (C.c_void_p * P)(*[t.data_ptr() for t in us])
    pa = (C.c_void_p * P)(*[t.data_ptr() for t in ps])
    sts = (stp_stats * P)()
    status = load().stp_uzawa_solve_batch(ctx, ua, pa, sts)
    return status, list(sts)


def stp_batch_size(ctx) -> int:
    return int(load().stp_batch_size(ctx))


def stp_apply_operator(ctx, op, x, y):
    _check(load().stp_apply_operator(ctx, op, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())),
           "stp_apply_operator")


def stp_apply_precond(ctx, which, r, z):
    _check(load().stp_apply_precond(ctx, which, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())),
           "stp_apply_precond")


def stp_uzawa_solve(ctx, u, p):
    st = stp_stats()
    status = load().stp_uzawa_solve(ctx, C.c_void_p(u.data_ptr()), C.c_void_p(p.data_ptr()), C.byref(st))
    return status, st


def stp_gmres_workspace_bytes(ctx, restart) -> int:
    return int(load().stp_gmres_workspace_bytes(ctx, int(restart)))


def stp_gmres_solve(ctx, u, p, restart, ws, max_iter=None):
    """GMRES(restart) around the Uzawa sweep; ws: a device tensor of at least
    stp_gmres_workspace_bytes bytes; max_iter: the context's (sizes the
    residual history; None: no history).  Returns (status, stats, history)."""
    st = stp_stats()
    hist = (C.c_double * (max_iter + 1))() if max_iter is not None else None
    status = load().stp_gmres_solve(ctx, C.c_void_p(u.data_ptr()), C.c_void_p(p.data_ptr()), int(restart),
                                    C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel() * ws.element_size()),
                                    hist, C.byref(st))
    h = None if hist is None else [hist[i] for i in range(st.iters + 1)]
    return status, st, h


def stp_gmres_solve_noalloc(ctx, u, p, restart, max_iter=None):
    """stp_gmres_solve with the library's fixed Krylov array (the call allocates
    no device memory).  Returns (status, stats, history)."""
    st = stp_stats()
    hist = (C.c_double * (max_iter + 1))() if max_iter is not None else None
    status = load().stp_gmres_solve_noalloc(ctx, C.c_void_p(u.data_ptr()), C.c_void_p(p.data_ptr()), int(restart),
                                            hist, C.byref(st))
    h = None if hist is None else [hist[i] for i in range(st.iters + 1)]
    return status, st, h


def stp_autotune(ctx, reps=5, use_cache=True):
    """Tune the launch schedule of the context; returns the report as a dict."""
    r = stp_tune_report()
    _check(load().stp_autotune(ctx, int(reps), 1 if use_cache else 0, C.byref(r)), "stp_autotune")
    return dict(knobs_tuned=r.knobs_tuned, candidates=r.candidates, from_cache=bool(r.from_cache),
                iter_ms_before=r.iter_ms_before, iter_ms_after=r.iter_ms_after)


def stp_omega_info(ctx, i=0):
    out = (C.c_double * 5)()
    _check(load().stp_omega_info(ctx, int(i), out), "stp_omega_info")
    return dict(omega=out[0], lmin=out[1], lmax=out[2], rho_A=out[3], omega_37=out[4])


def stp_device_bytes_allocated() -> int:
    return int(load().stp_device_bytes_allocated())


def stp_set_stop(ctx, tol, max_iter):
    _check(load().stp_set_stop(ctx, float(tol), int(max_iter)), "stp_set_stop")


def stp_set_omega(ctx, omegas):
    arr = (C.c_double * len(omegas))(*[float(w) for w in omegas])
    _check(load().stp_set_omega(ctx, arr), "stp_set_omega")


def stp_schedule_string(ctx) -> str:
    return load().stp_schedule_string(ctx).decode()


def stp_timing_enable(ctx, enable=True):
    _check(load().stp_timing_enable(ctx, 1 if enable else 0), "stp_timing_enable")


def stp_timing_report(ctx):
    """List of dicts (kernel, level, launches, total_ms, avg_ms) since stp_timing_enable."""
    lib = load()
    n = lib.stp_timing_count(ctx)
    if n < 0:
        _check(STP_EDEVICE, "stp_timing_count")
    out = []
    for i in range(n):
        name, lev, cnt, ms = C.c_char_p(), C.c_int(), C.c_long(), C.c_double()
        _check(lib.stp_timing_get(ctx, i, C.byref(name), C.byref(lev), C.byref(cnt), C.byref(ms)), "stp_timing_get")
        kern = name.value.decode().strip("()")
        out.append(dict(kernel=kern, level=lev.value, launches=cnt.value, total_ms=ms.value,
                        avg_ms=ms.value / max(cnt.value, 1)))
    return out


def stp_destroy(ctx):
    if ctx:
        load().stp_destroy(ctx)


# --- convenience wrapper ------------------------------------------------------------

class SpaceTimeSolver:
    """One problem on one GPU.  Tensors are float64 CUDA tensors laid out as in stp.h."""

    def __init__(self, dim, n, N, tau, kfields, tcoef, F, u0, stream=None, workspace=None, **opts):
        import torch
        self.dim, self.n, self.N = dim, n, N
        self.shape = (N,) + (n,) * dim
        self.device = F.device
        self.stream = stream
        self.max_iter = int(opts.get("max_iter", 500))
        with torch.cuda.device(self.device):
            self.ctx, self._keep = stp_create(dim, n, N, tau, kfields, tcoef, F, u0,
                                              workspace=workspace, stream=stream, **opts)

    def _vec(self, x, k=1):
        shape = (k,) + self.shape if k > 1 else self.shape
        _dev_f64(x, shape, "vector")
        return x

    def apply_operator(self, op, x, y=None):
        import torch
        k = 2 if op == STP_OP_SADDLE else 1
        self._vec(x, k)
        y = torch.empty_like(x) if y is None else self._vec(y, k)
        stp_apply_operator(self.ctx, op, x, y)
        return y

    def apply_precond(self, which, r, z=None):
        import torch
        self._vec(r)
        z = torch.empty_like(r) if z is None else self._vec(z)
        stp_apply_precond(self.ctx, which, r, z)
        return z

    def solve(self, u=None, p=None, raise_on_error=False):
        """Run the Uzawa iteration from (u, p) (zeros if None).  Returns (u, p, stats dict)."""
        import torch
        u = torch.zeros(self.shape, dtype=torch.float64, device=self.device) if u is None else self._vec(u)
        p = torch.zeros(self.shape, dtype=torch.float64, device=self.device) if p is None else self._vec(p)
        status, st = stp_uzawa_solve(self.ctx, u, p)
        info = stats_dict(st, status)
        if raise_on_error and status != STP_OK:
            _check(status, "stp_uzawa_solve")
        if status not in (STP_OK, STP_ENOTCONV, STP_EDIVERGED):
            _check(status, "stp_uzawa_solve")
        return u, p, info

    def gmres(self, u=None, p=None, restart=20, workspace=None, raise_on_error=False):
        """GMRES(restart) acceleration of the Uzawa sweep from (u, p) (zeros if
        None), with the context's tol, max_iter and omega.  Returns (u, p,
        stats dict with the residual history)."""
        import torch
        u = torch.zeros(self.shape, dtype=torch.float64, device=self.device) if u is None else self._vec(u)
        p = torch.zeros(self.shape, dtype=torch.float64, device=self.device) if p is None else self._vec(p)
        nb = stp_gmres_workspace_bytes(self.ctx, restart)
        if nb == 0:
            raise StpError(STP_EINVAL, f"no GMRES workspace size for restart {restart}")
        if workspace is None or workspace.numel() * workspace.element_size() < nb:
            workspace = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        status, st, hist = stp_gmres_solve(self.ctx, u, p, restart, workspace, self.max_iter)
        info = stats_dict(st, status)
        info["history"] = hist
        if raise_on_error and status != STP_OK:
            _check(status, "stp_gmres_solve")
        if status not in (STP_OK, STP_ENOTCONV, STP_EDIVERGED):
            _check(status, "stp_gmres_solve")
        return u, p, info

    def timing(self, enable=True):
        stp_timing_enable(self.ctx, enable)

    def timing_report(self):
        return stp_timing_report(self.ctx)

    def autotune(self, reps=5, use_cache=True):
        return stp_autotune(self.ctx, reps, use_cache)

    def schedule(self):
        return stp_schedule_string(self.ctx)

    def omega_info(self, i=0):
        return stp_omega_info(self.ctx, i)

    def set_stop(self, tol, max_iter):
        """Stop rule of the following solves (the captured iteration graph stays valid)."""
        stp_set_stop(self.ctx, tol, max_iter)
        self.max_iter = int(max_iter)

    def close(self):
        if self.ctx:
            stp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Many independent problems of one spatial dimension in one context: every
    step of an iteration is a merged launch over the whole batch."""

    def __init__(self, problems, stream=None, workspace=None, **opts):
        import torch
        self.shapes = [(q["N"],) + (q["n"],) * q["dim"] for q in problems]
        self.device = problems[0]["F"].device
        with torch.cuda.device(self.device):
            self.ctx, self._keep = stp_create_batch(problems, workspace=workspace, stream=stream, **opts)

    def __len__(self):
        return len(self.shapes)

    def omegas(self):
        return [stp_omega_info(self.ctx, i)["omega"] for i in range(len(self.shapes))]

    def set_omegas(self, omegas):
        stp_set_omega(self.ctx, omegas)

    def set_stop(self, tol, max_iter):
        """Stop rule of the following solves of every problem."""
        stp_set_stop(self.ctx, tol, max_iter)

    def solve(self, us=None, ps=None):
        """Solve every problem from (us[i], ps[i]) (zeros if None).  Returns (us, ps, infos, status)."""
        import torch
        z = lambda sh: torch.zeros(sh, dtype=torch.float64, device=self.device)  # noqa: E731
        us = [z(sh) for sh in self.shapes] if us is None else list(us)
        ps = [z(sh) for sh in self.shapes] if ps is None else list(ps)
        for i, sh in enumerate(self.shapes):
            _dev_f64(us[i], sh, f"u[{i}]")
            _dev_f64(ps[i], sh, f"p[{i}]")
        status, sts = stp_uzawa_solve_batch(self.ctx, us, ps)
        if status not in (STP_OK, STP_ENOTCONV, STP_EDIVERGED):
            _check(status, "stp_uzawa_solve_batch")
        infos = [stats_dict(s) for s in sts]
        return us, ps, infos, status

    def timing(self, enable=True):
        stp_timing_enable(self.ctx, enable)

    def timing_report(self):
        return stp_timing_report(self.ctx)

    def autotune(self, reps=5, use_cache=True):
        return stp_autotune(self.ctx, reps, use_cache)

    def schedule(self):
        return stp_schedule_string(self.ctx)

    def omega_info(self, i=0):
        return stp_omega_info(self.ctx, i)

    def close(self):
        if self.ctx:
            stp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def problem_dict(prob, device="cuda"):
    """Device copy of a ``synth.Problem`` in the form stp_create_batch takes."""
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)  # noqa: E731
    d = dict(dim=prob.dim, n=prob.n, N=prob.N, tau=prob.tau, kfields=t(prob.kfields), tcoef=prob.tcoef,
             F=t(prob.F), u0=t(prob.u0))
    if getattr(prob, "steps", None) is not None:
        d["steps"] = list(prob.steps)
    return d


def from_problem(prob, device="cuda", **opts):
    """Build a solver from a ``synth.Problem`` (copies its arrays to the device;
    its step lengths, when non-uniform, become the tau_steps option)."""
    import torch
    kf = torch.as_tensor(np.ascontiguousarray(prob.kfields), dtype=torch.float64, device=device)
    F = torch.as_tensor(np.ascontiguousarray(prob.F), dtype=torch.float64, device=device)
    u0 = torch.as_tensor(np.ascontiguousarray(prob.u0), dtype=torch.float64, device=device)
    if getattr(prob, "steps", None) is not None and "tau_steps" not in opts:
        opts["tau_steps"] = list(prob.steps)
    return SpaceTimeSolver(prob.dim, prob.n, prob.N, prob.tau, kf, prob.tcoef, F, u0, **opts)
