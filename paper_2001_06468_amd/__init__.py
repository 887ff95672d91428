"""Python binding of libnrs, the MI355X (gfx950) implementation of the
nearest-neighbour regularized stokeslet hot path (Gallagher & Smith,
arXiv:2001.06468).

Every function mirrors the C entry point of the same name in include/nrs.h
and only marshals arguments: torch tensors supply device memory, the current
torch stream supplies the HIP stream, and all arithmetic runs in the HIP
kernels of libnrs.so.  Nothing here falls back to a CPU implementation: if
the library is missing or a tensor is not on the GPU the call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (NRS_BF16_GMRES_IR, NRS_FP32_GEPP_IR, NRS_FP32_GMRES_IR, NRS_FP32_IR,  # noqa: F401
                   NRS_FP64_LU,
                   NRS_GMRES, NRS_GMRES_BLOCK, NRS_PRECOND_EXACT, NRS_PRECOND_MODEL,
                   NRS_BLOCK_MAX_HARMONICS,
                   NRS_MLP_HIDDEN, NRS_MLP_MAX_POINTS, NRS_NOALLOC_MAX_N, NRS_WARM_MODEL, NRS_WARM_NONE,
                   NRS_WARM_PREVIOUS, NrsInfo, NrsOptions, NrsProblem, NrsScene)

__all__ = [
    "NrsError", "Context", "DeviceScene", "Problem", "nrs_create", "nrs_version", "nrs_geometry",
    "nrs_nearest", "nrs_workspace_size", "nrs_assemble", "nrs_apply", "nrs_solve",
    "nrs_query_info", "nrs_solve_batched_workspace_size", "nrs_solve_batched", "nrs_lu_factor", "nrs_lu_solve",
    "nrs_lu_factor_workspace_size", "nrs_lu_solve_workspace_size", "nrs_lu_query", "nrs_lu_solve_noalloc", "nrs_equilibrate", "nrs_rk4_workspace_size", "nrs_rk4_step",
    "NRS_FP64_LU", "NRS_FP32_IR", "NRS_FP32_GEPP_IR", "NRS_GMRES", "NRS_FP32_GMRES_IR", "NRS_BF16_GMRES_IR",
    "lda_for",
    "NRS_WARM_NONE", "NRS_WARM_PREVIOUS", "NRS_WARM_MODEL", "Model", "nrs_mlp_param_count",
    "nrs_autotune", "nrs_autotune_clear",
    "nrs_mlp_body_offsets", "nrs_mlp_features", "nrs_mlp_forward", "nrs_mlp_grad",
    "nrs_mlp_grad_workspace_size", "nrs_adam_step", "nrs_mlp_targets",
    "nrs_mlp_warm_start_workspace_size", "nrs_mlp_warm_start", "nrs_mlp_status",
    "nrs_field_workspace_size", "nrs_field_velocity", "nrs_tracer_rk4_step",
    "nrs_rk4_tracers_workspace_size", "nrs_rk4_step_tracers",
    "nrs_dopri5_workspace_size", "nrs_dopri5_integrate",
    "NRS_GMRES_BLOCK", "NRS_PRECOND_EXACT", "NRS_PRECOND_MODEL", "NRS_BLOCK_MAX_HARMONICS",
    "BlockModel", "nrs_block_limit", "nrs_block_invert", "nrs_block_model_fit",
    "nrs_block_model_eval",
]


class NrsError(RuntimeError):
    def __init__(self, status, detail=""):
        lib = _lib.load()
        super().__init__(f"{lib.nrs_status_string(status).decode()} ({status}): {detail}")
        self.status = status


def _check(status, ctx=None):
    if status != 0:
        detail = ""
        if ctx is not None:
            detail = _lib.load().nrs_last_error(ctx.handle).decode(errors="replace")
        raise NrsError(status, detail)


def _ptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def lda_for(n):
    """Leading dimension the library uses for its own matrices (multiple of 64)."""
    return max(64, (n + 63) // 64 * 64)


def nrs_version():
    return _lib.load().nrs_version().decode()


class Context:
    """Owns an nrs_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device=0, stream=None):
        lib = _lib.load()
        self.device = device
        h = C.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        _check(lib.nrs_create(C.byref(h), device, C.c_void_p(stream)))
        self.handle = h

    def set_stream(self, stream):
        _check(_lib.load().nrs_set_stream(self.handle, C.c_void_p(stream)), self)

    def close(self):
        if self.handle:
            _lib.load().nrs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nrs_create(device=0, stream=None):
    return Context(device, stream)


class DeviceScene:
    """Device copy of a scene description (see the ``synth`` package for the
    field meanings); exposes the nrs_scene struct of include/nrs.h."""

    _F64 = ("xi", "s", "ufix", "Xi", "sX", "w0", "wave", "Y0", "ftext")
    _I32 = ("body", "part", "bodyX", "partX", "groupX")

    def __init__(self, scene, device="cuda"):
        self.N, self.Q, self.M = int(scene["N"]), int(scene["Q"]), int(scene["M"])
        self.eps, self.mu = float(scene["eps"]), float(scene["mu"])
        self.group_off = np.ascontiguousarray(scene["group_off"], dtype=np.int32)
        self.G = len(self.group_off) - 1
        self.t = {}
        for k in self._F64:
            a = np.ascontiguousarray(scene[k], dtype=np.float64)
            self.t[k] = torch.from_numpy(a.copy()).to(device)
        for k in self._I32:
            a = np.ascontiguousarray(scene[k], dtype=np.int32)
            self.t[k] = torch.from_numpy(a.copy()).to(device)
        self.P = int(self.t["wave"].shape[0])

    def struct(self):
        t = self.t
        return NrsScene(self.N, self.Q, self.M, self.P,
                        _ptr(t["xi"]), _ptr(t["body"]), _ptr(t["part"]), _ptr(t["s"]),
                        _ptr(t["ufix"]), _ptr(t["Xi"]), _ptr(t["bodyX"]), _ptr(t["partX"]),
                        _ptr(t["sX"]), _ptr(t["w0"]), _ptr(t["wave"]) if self.P else None)


class Problem:
    """Tensors of one nrs_problem (device memory)."""

    def __init__(self, x, X, w, nu, body, Y, eps, mu):
        self.x, self.X, self.w, self.nu, self.body, self.Y = x, X, w, nu, body, Y
        self.N = int(x.shape[-1])
        self.Q = int(X.shape[-1])
        self.M = 0 if Y is None else int(Y.reshape(-1, 12).shape[0])
        self.eps, self.mu = float(eps), float(mu)

    @property
    def n(self):
        return 3 * self.N + 6 * self.M

    def struct(self):
        f64, i32 = torch.float64, torch.int32
        return NrsProblem(self.N, self.Q, self.M, _ptr(self.x, f64, "x"), _ptr(self.X, f64, "X"),
                          _ptr(self.w, f64, "w"), _ptr(self.nu, i32, "nu"),
                          _ptr(self.body, i32, "body"), _ptr(self.Y, f64, "Y"),
                          self.eps, self.mu)


class Model:
    """Parameters of the warm-start network (device FP32 [nrs_mlp_param_count()])
    and the (force, U, Omega) scales of its outputs."""

    def __init__(self, theta, scales):
        if theta.dtype != torch.float32 or theta.numel() != nrs_mlp_param_count():
            raise ValueError("theta must be float32 with nrs_mlp_param_count() entries")
        self.theta = theta
        self.scales = tuple(float(v) for v in scales)


class BlockModel:
    """Learned body-block inverse of NRS_GMRES_BLOCK: device FP64 model
    [2H+1][nb][nb] (each block column-major, i.e. the torch view of a block
    is its transpose) from nrs_block_model_fit, harmonics H, order nb."""

    def __init__(self, coef, nb, H):
        if coef.dtype != torch.float64 or tuple(coef.shape) != (2 * H + 1, nb, nb):
            raise ValueError("coef must be float64 of shape (2H+1, nb, nb)")
        self.coef, self.nb, self.H = coef, int(nb), int(H)


def _options(method=NRS_FP64_LU, max_refine=0, tol=0.0, gmres_restart=0, gmres_max_iter=0,
             no_fallback=0, x_init=None, warm_start=NRS_WARM_NONE, model=None, body_off=None,
             x_init_complete=0, graph=0, reuse_stage_factors=0, equilibrate=0,
             precond=NRS_PRECOND_EXACT, block_model=None, precond_phase=None, ir_queue=0):
    sc = (C.c_double * 3)(*(model.scales if model is not None else (0.0, 0.0, 0.0)))
    bm = block_model
    return NrsOptions(method, max_refine, tol, gmres_restart, gmres_max_iter, no_fallback,
                      _ptr(x_init, torch.float64, "x_init"), warm_start,
                      _ptr(model.theta, torch.float32, "theta") if model is not None else None,
                      sc, _ptr(body_off, torch.int32, "body_off"), int(x_init_complete),
                      int(graph), int(reuse_stage_factors), int(equilibrate), int(precond),
                      bm.H if bm is not None else 0, bm.nb if bm is not None else 0,
                      _ptr(bm.coef, torch.float64, "block model") if bm is not None else None,
                      _ptr(precond_phase, torch.float64, "precond_phase"), int(ir_queue))


def nrs_geometry(ctx, scene, t, Y, x=None, X=None, w=None, u=None):
    f64 = torch.float64
    sc = scene.struct()
    _check(_lib.load().nrs_geometry(ctx.handle, C.byref(sc), float(t), _ptr(Y, f64, "Y"),
                                    _ptr(x, f64, "x"), _ptr(X, f64, "X"), _ptr(w, f64, "w"),
                                    _ptr(u, f64, "u")), ctx)


def nrs_nearest(ctx, x, group_off, X, groupX, nu_out):
    go = np.ascontiguousarray(group_off, dtype=np.int32)
    _check(_lib.load().nrs_nearest(ctx.handle, int(x.shape[-1]), _ptr(x, torch.float64, "x"),
                                   len(go) - 1, go.ctypes.data_as(C.c_void_p), int(X.shape[-1]),
                                   _ptr(X, torch.float64, "X"), _ptr(groupX, torch.int32, "groupX"),
                                   _ptr(nu_out, torch.int32, "nu_out")), ctx)


def nrs_workspace_size(ctx, N, Q, M, method):
    b = C.c_size_t()
    _check(_lib.load().nrs_workspace_size(ctx.handle, N, Q, M, method, C.byref(b)), ctx)
    return b.value


def nrs_assemble(ctx, problem, precision, A, lda, ws):
    dt = torch.float32 if precision == 32 else torch.float64
    pb = problem.struct()
    _check(_lib.load().nrs_assemble(ctx.handle, C.byref(pb), precision, _ptr(A, dt, "A"), lda,
                                    _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)


def nrs_apply(ctx, problem, v, y, ws):
    pb = problem.struct()
    _check(_lib.load().nrs_apply(ctx.handle, C.byref(pb), _ptr(v, torch.float64, "v"),
                                 _ptr(y, torch.float64, "y"), _ptr(ws, torch.uint8, "ws"),
                                 ws.numel()), ctx)


def nrs_solve(ctx, problem, u, ftext, sol, ws, method=NRS_FP64_LU, info=True, **opts):
    """Returns the nrs_info dict (synchronising) or None (asynchronous)."""
    pb = problem.struct()
    o = _options(method, **opts)
    inf = NrsInfo() if info else None
    st = _lib.load().nrs_solve(ctx.handle, C.byref(pb), _ptr(u, torch.float64, "u"),
                               _ptr(ftext, torch.float64, "ftext"), C.byref(o),
                               _ptr(ws, torch.uint8, "ws"), ws.numel(),
                               _ptr(sol, torch.float64, "sol"),
                               C.byref(inf) if inf is not None else None)
    _check(st, ctx)
    return inf.as_dict() if inf is not None else None


def _problem_array(problems):
    arr = (NrsProblem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p.struct()
    return arr


def nrs_solve_batched_workspace_size(ctx, problems, method=NRS_FP32_IR):
    b = C.c_size_t()
    arr = _problem_array(problems)
    _check(_lib.load().nrs_solve_batched_workspace_size(ctx.handle, len(problems), arr, method,
                                                        C.byref(b)), ctx)
    return b.value


def nrs_solve_batched(ctx, problems, us, sols, ws, ftexts=None, method=NRS_FP32_IR, info=True,
                      **opts):
    """Returns a list of nrs_info dicts (synchronising) or None (asynchronous)."""
    B = len(problems)
    if len(us) != B or len(sols) != B or (ftexts is not None and len(ftexts) != B):
        raise ValueError("problems, us, sols (and ftexts) need the same length")
    arr = _problem_array(problems)
    f64 = torch.float64
    u_p = (C.c_void_p * B)(*[_ptr(u, f64, "u") for u in us])
    s_p = (C.c_void_p * B)(*[_ptr(x, f64, "sol") for x in sols])
    f_p = None
    if ftexts is not None:
        f_p = (C.c_void_p * B)(*[_ptr(f, f64, "ftext") for f in ftexts])
    o = _options(method, **opts)
    infs = (NrsInfo * B)() if info else None
    st = _lib.load().nrs_solve_batched(ctx.handle, B, arr, u_p, f_p, C.byref(o),
                                       _ptr(ws, torch.uint8, "ws"), ws.numel(), s_p, infs)
    _check(st, ctx)
    return [i.as_dict() for i in infs] if infs is not None else None


def nrs_query_info(ctx, ws):
    inf = NrsInfo()
    _check(_lib.load().nrs_query_info(ctx.handle, _ptr(ws, torch.uint8, "ws"), C.byref(inf)), ctx)
    return inf.as_dict()


def _lu_prec(A, bf16_updates=False):
    prec = 32 if A.dtype == torch.float32 else 64
    if bf16_updates:
        if prec != 32:
            raise TypeError("BF16 updates need an FP32 matrix")
        prec = 16
    return prec


def nrs_lu_factor_workspace_size(ctx, n, precision):
    b = C.c_size_t()
    _check(_lib.load().nrs_lu_factor_workspace_size(ctx.handle, n, precision, C.byref(b)), ctx)
    return b.value


def nrs_lu_solve_workspace_size(ctx, n):
    b = C.c_size_t()
    _check(_lib.load().nrs_lu_solve_workspace_size(ctx.handle, n, C.byref(b)), ctx)
    return b.value


def nrs_lu_factor(ctx, A, lda, ipiv, perm, singular, ws, pivot_scope=0, bf16_updates=False):
    """bf16_updates (FP32 A, pivot_scope 1): trailing updates on BF16 tile copies.
    ws: uint8 device tensor of nrs_lu_factor_workspace_size bytes."""
    prec = _lu_prec(A, bf16_updates)
    n = int(ipiv.numel())
    _check(_lib.load().nrs_lu_factor(ctx.handle, n, prec, pivot_scope, _ptr(A, A.dtype, "A"), lda,
                                     _ptr(ipiv, torch.int32, "ipiv"), _ptr(perm, torch.int32, "perm"),
                                     _ptr(singular, torch.int32, "singular"),
                                     _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)


def nrs_lu_solve(ctx, LU, lda, perm, b, x, ws, pivot_scope=0):
    """ws: uint8 device tensor of nrs_lu_solve_workspace_size bytes."""
    prec = 32 if LU.dtype == torch.float32 else 64
    n = int(perm.numel())
    _check(_lib.load().nrs_lu_solve(ctx.handle, n, prec, pivot_scope, _ptr(LU, LU.dtype, "LU"), lda,
                                    _ptr(perm, torch.int32, "perm"), _ptr(b, LU.dtype, "b"),
                                    _ptr(x, LU.dtype, "x"), _ptr(ws, torch.uint8, "ws"),
                                    ws.numel()), ctx)


def nrs_lu_solve_noalloc(ctx, LU, lda, perm, b, x, pivot_scope=0):
    """nrs_lu_solve on the library's static scratch (no workspace, no allocation)."""
    prec = 32 if LU.dtype == torch.float32 else 64
    n = int(perm.numel())
    _check(_lib.load().nrs_lu_solve_noalloc(ctx.handle, n, prec, pivot_scope,
                                            _ptr(LU, LU.dtype, "LU"), lda,
                                            _ptr(perm, torch.int32, "perm"), _ptr(b, LU.dtype, "b"),
                                            _ptr(x, LU.dtype, "x")), ctx)


def nrs_equilibrate(ctx, A, lda, dr, dc, ws):
    """A (FP32, column-major as [n][lda]) <- D_r A D_c in place; dr, dc: [n] FP32."""
    n = int(dr.numel())
    f32 = torch.float32
    _check(_lib.load().nrs_equilibrate(ctx.handle, n, _ptr(A, f32, "A"), lda, _ptr(dr, f32, "dr"),
                                       _ptr(dc, f32, "dc"), _ptr(ws, torch.uint8, "ws"),
                                       ws.numel()), ctx)


def nrs_lu_query(ctx, ws=None):
    """ws = None: the last nrs_lu_solve_noalloc on the context's device."""
    f = C.c_int32()
    _check(_lib.load().nrs_lu_query(ctx.handle, _ptr(ws, torch.uint8, "ws"), C.byref(f)), ctx)
    return f.value


def nrs_rk4_workspace_size(ctx, scene, method):
    b = C.c_size_t()
    sc = scene.struct()
    _check(_lib.load().nrs_rk4_workspace_size(ctx.handle, C.byref(sc), method, C.byref(b)), ctx)
    return b.value


def nrs_rk4_step(ctx, scene, Y, t, dt, ws, method=NRS_FP64_LU, ftext=None, **opts):
    sc = scene.struct()
    o = _options(method, **opts)
    go = scene.group_off
    _check(_lib.load().nrs_rk4_step(ctx.handle, C.byref(sc), len(go) - 1,
                                    go.ctypes.data_as(C.c_void_p),
                                    _ptr(scene.t["groupX"], torch.int32, "groupX"), scene.eps,
                                    scene.mu, _ptr(ftext, torch.float64, "ftext"),
                                    _ptr(Y, torch.float64, "Y"), float(t), float(dt), C.byref(o),
                                    _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)


def nrs_rk4_tracers_workspace_size(ctx, scene, method, P):
    b = C.c_size_t()
    sc = scene.struct()
    _check(_lib.load().nrs_rk4_tracers_workspace_size(ctx.handle, C.byref(sc), method, int(P),
                                                      C.byref(b)), ctx)
    return b.value


def nrs_rk4_step_tracers(ctx, scene, Y, ytr, t, dt, ws, method=NRS_FP64_LU, ftext=None, **opts):
    """ytr: device float64 [3, P] tracer positions, advanced in place."""
    sc = scene.struct()
    o = _options(method, **opts)
    go = scene.group_off
    P = 0 if ytr is None else int(ytr.numel() // 3)
    _check(_lib.load().nrs_rk4_step_tracers(
        ctx.handle, C.byref(sc), len(go) - 1, go.ctypes.data_as(C.c_void_p),
        _ptr(scene.t["groupX"], torch.int32, "groupX"), scene.eps, scene.mu,
        _ptr(ftext, torch.float64, "ftext"), _ptr(Y, torch.float64, "Y"), float(t), float(dt),
        C.byref(o), P, _ptr(ytr, torch.float64, "ytr"), _ptr(ws, torch.uint8, "ws"),
        ws.numel()), ctx)


def nrs_dopri5_workspace_size(ctx, scene, method):
    b = C.c_size_t()
    sc = scene.struct()
    _check(_lib.load().nrs_dopri5_workspace_size(ctx.handle, C.byref(sc), method, C.byref(b)), ctx)
    return b.value


def nrs_dopri5_integrate(ctx, scene, Y, t0, t1, h, rtol, atol, ws, method=NRS_FP64_LU,
                         ftext=None, max_steps=100000, **opts):
    """Adaptive Dormand-Prince 5(4) from t0 to t1 (Y advanced in place);
    returns the stats dict (accepted, rejected, solves, fell_back, t, h)."""
    sc = scene.struct()
    o = _options(method, **opts)
    go = scene.group_off
    hh = C.c_double(float(h))
    st = _lib.NrsDopriStats()
    _check(_lib.load().nrs_dopri5_integrate(
        ctx.handle, C.byref(sc), len(go) - 1, go.ctypes.data_as(C.c_void_p),
        _ptr(scene.t["groupX"], torch.int32, "groupX"), scene.eps, scene.mu,
        _ptr(ftext, torch.float64, "ftext"), _ptr(Y, torch.float64, "Y"), float(t0), float(t1),
        C.byref(hh), float(rtol), float(atol), C.byref(o), int(max_steps), C.byref(st),
        _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)
    return st.as_dict()


# ---------------------------------------------------------------- field points and tracers

def nrs_field_workspace_size(ctx, P, Q):
    b = C.c_size_t()
    _check(_lib.load().nrs_field_workspace_size(ctx.handle, int(P), int(Q), C.byref(b)), ctx)
    return b.value


def nrs_field_velocity(ctx, problem, f, y, u, ws):
    """u [3, P] = flow of force densities f [3, N] at field points y [3, P]."""
    pb = problem.struct()
    P = int(y.numel() // 3)
    _check(_lib.load().nrs_field_velocity(ctx.handle, C.byref(pb), _ptr(f, torch.float64, "f"), P,
                                          _ptr(y, torch.float64, "y"),
                                          _ptr(u, torch.float64, "u"),
                                          _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)


def nrs_tracer_rk4_step(ctx, problems, fs, y, dt, ws):
    """problems, fs: the flows (Problem) and force densities at t, t + dt/2,
    t + dt; y [3, P] advanced in place."""
    if len(problems) != 3 or len(fs) != 3:
        raise ValueError("three flows (t, t + dt/2, t + dt) required")
    arr = (NrsProblem * 3)(*[p.struct() for p in problems])
    fp = (C.c_void_p * 3)(*[_ptr(f, torch.float64, "f") for f in fs])
    P = int(y.numel() // 3)
    _check(_lib.load().nrs_tracer_rk4_step(ctx.handle, arr, fp, P, _ptr(y, torch.float64, "y"),
                                           float(dt), _ptr(ws, torch.uint8, "ws"), ws.numel()),
           ctx)


# ---------------------------------------------------------------- learned warm start

def nrs_mlp_param_count():
    return int(_lib.load().nrs_mlp_param_count())


def nrs_mlp_body_offsets(ctx, body, M):
    """Device int32 [M+1] offsets of each body's contiguous run of points."""
    off = torch.empty(M + 1, dtype=torch.int32, device=body.device)
    _check(_lib.load().nrs_mlp_body_offsets(ctx.handle, body.numel(), _ptr(body, torch.int32, "body"),
                                            M, _ptr(off, torch.int32, "body_off")), ctx)
    return off


def nrs_mlp_features(ctx, x, u, s, body, M, Y, phi):
    f64 = torch.float64
    _check(_lib.load().nrs_mlp_features(ctx.handle, body.numel(), _ptr(x, f64, "x"), _ptr(u, f64, "u"),
                                        _ptr(s, f64, "s"), _ptr(body, torch.int32, "body"), M,
                                        _ptr(Y, f64, "Y"), _ptr(phi, torch.float32, "phi")), ctx)


def nrs_mlp_forward(ctx, theta, M, body_off, phi, y, z, sel=None):
    f32 = torch.float32
    nsel = 0 if sel is None else sel.numel()
    _check(_lib.load().nrs_mlp_forward(ctx.handle, _ptr(theta, f32, "theta"), phi.shape[0], M,
                                       _ptr(body_off, torch.int32, "body_off"),
                                       _ptr(sel, torch.int32, "sel"), nsel, _ptr(phi, f32, "phi"),
                                       _ptr(y, f32, "y"), _ptr(z, f32, "z")), ctx)


def nrs_mlp_grad_workspace_size(nsel):
    b = C.c_size_t()
    _check(_lib.load().nrs_mlp_grad_workspace_size(nsel, C.byref(b)))
    return b.value


def nrs_mlp_grad(ctx, theta, M, body_off, phi, t_pt, t_body, grad, ws, sel=None):
    """grad: float32 [nrs_mlp_param_count() + 1]; the last entry receives the loss."""
    f32 = torch.float32
    nsel = 0 if sel is None else sel.numel()
    _check(_lib.load().nrs_mlp_grad(ctx.handle, _ptr(theta, f32, "theta"), phi.shape[0], M,
                                    _ptr(body_off, torch.int32, "body_off"),
                                    _ptr(sel, torch.int32, "sel"), nsel, _ptr(phi, f32, "phi"),
                                    _ptr(t_pt, f32, "t_pt"), _ptr(t_body, f32, "t_body"),
                                    _ptr(grad, f32, "grad"), _ptr(ws, torch.uint8, "ws"),
                                    ws.numel()), ctx)


def nrs_adam_step(ctx, theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    f32 = torch.float32
    _check(_lib.load().nrs_adam_step(ctx.handle, theta.numel(), _ptr(theta, f32, "theta"),
                                     _ptr(grad, f32, "grad"), _ptr(m, f32, "m"), _ptr(v, f32, "v"),
                                     int(step), float(lr), float(beta1), float(beta2), float(eps)),
           ctx)


def nrs_mlp_targets(ctx, body, M, Y, sol, scales, t_pt, t_body):
    f64 = torch.float64
    sc = (C.c_double * 3)(*scales)
    _check(_lib.load().nrs_mlp_targets(ctx.handle, body.numel(), M, _ptr(body, torch.int32, "body"),
                                       _ptr(Y, f64, "Y"), _ptr(sol, f64, "sol"), sc,
                                       _ptr(t_pt, torch.float32, "t_pt"),
                                       _ptr(t_body, torch.float32, "t_body")), ctx)


def nrs_mlp_warm_start_workspace_size(N, M):
    b = C.c_size_t()
    _check(_lib.load().nrs_mlp_warm_start_workspace_size(N, M, C.byref(b)))
    return b.value


def nrs_mlp_warm_start(ctx, model, body, body_off, x, u, s, Y, x0, ws):
    f64 = torch.float64
    M = body_off.numel() - 1
    sc = (C.c_double * 3)(*model.scales)
    _check(_lib.load().nrs_mlp_warm_start(ctx.handle, _ptr(model.theta, torch.float32, "theta"), sc,
                                          body.numel(), M, _ptr(body, torch.int32, "body"),
                                          _ptr(body_off, torch.int32, "body_off"),
                                          _ptr(x, f64, "x"), _ptr(u, f64, "u"), _ptr(s, f64, "s"),
                                          _ptr(Y, f64, "Y"), _ptr(x0, f64, "x0"),
                                          _ptr(ws, torch.uint8, "ws"), ws.numel()), ctx)


def nrs_mlp_status(ctx):
    f = C.c_int32()
    _check(_lib.load().nrs_mlp_status(ctx.handle, C.byref(f)), ctx)
    return f.value


# ---------------------------------------------------------------- autotuning

def nrs_autotune(ctx, problem, ws):
    """Tune the assembly launch shape for the problem's size class; returns the
    choice and timings (dict)."""
    pb = problem.struct()
    out = _lib.NrsTuneResult()
    _check(_lib.load().nrs_autotune(ctx.handle, C.byref(pb), _ptr(ws, torch.uint8, "ws"),
                                    ws.numel(), C.byref(out)), ctx)
    return out.as_dict()


def nrs_block_limit(ctx):
    v = C.c_int32()
    _check(_lib.load().nrs_block_limit(ctx.handle, C.byref(v)), ctx)
    return v.value


def nrs_block_invert(ctx, blocks, singular):
    """blocks: float64 [count, nb, nb] (column-major blocks: blocks[i] is the
    transpose of block i), inverted in place; singular: int32 [1]."""
    count, nb = int(blocks.shape[0]), int(blocks.shape[-1])
    _check(_lib.load().nrs_block_invert(ctx.handle, count, nb, _ptr(blocks, torch.float64, "blocks"),
                                        _ptr(singular, torch.int32, "singular")), ctx)


def nrs_block_model_fit(ctx, inverses, H, model):
    """inverses: float64 [S, nb, nb]; model: float64 [2H+1, nb, nb] output."""
    S, nb = int(inverses.shape[0]), int(inverses.shape[-1])
    _check(_lib.load().nrs_block_model_fit(ctx.handle, S, nb, int(H),
                                           _ptr(inverses, torch.float64, "inverses"),
                                           _ptr(model, torch.float64, "model")), ctx)


def nrs_block_model_eval(ctx, model, H, psi, blocks):
    nb = int(model.shape[-1])
    _check(_lib.load().nrs_block_model_eval(ctx.handle, nb, int(H), _ptr(model, torch.float64, "model"),
                                            int(psi.numel()), _ptr(psi, torch.float64, "psi"),
                                            _ptr(blocks, torch.float64, "blocks")), ctx)


def nrs_autotune_clear(ctx):
    _check(_lib.load().nrs_autotune_clear(ctx.handle), ctx)
