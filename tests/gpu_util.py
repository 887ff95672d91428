"""Shared helpers of the GPU parity tests: upload seeded oracle-side inputs
and call the HIP path through the C ABI binding."""
import numpy as np
import torch

import oracle
import paper_2001_06468_amd as nrs

DEV = "cuda"


def T(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device=DEV)


def prepare(scene, t=0.0, Y=None):
    """Oracle-side geometry and nearest map of a scene state, plus the device
    Problem fed with exactly the same arrays."""
    Y = scene["Y0"] if Y is None else Y
    x, X, w, u = oracle.geometry(scene, t, Y)
    nu = oracle.nearest(x, X, scene["group_off"], scene["groupX"])
    pb = nrs.Problem(T(x), T(X), T(w), T(nu, torch.int32), T(scene["body"], torch.int32),
                     T(Y) if scene["M"] else None, scene["eps"], scene["mu"])
    host = dict(x=x, X=X, w=w, u=u, nu=nu, Y=Y)
    return pb, host


def oracle_system(scene, host):
    N, M = scene["N"], scene["M"]
    As = oracle.assemble_As(host["x"], host["X"], host["w"], host["nu"], scene["eps"], scene["mu"])
    W = oracle.patch_weights(host["w"], host["nu"], N)
    A = oracle.assemble_system(As, host["x"], W, scene["body"], host["Y"], M)
    b = oracle.rhs(host["u"], scene["ftext"])
    return A, b


def workspace(ctx, pb, method):
    nbytes = nrs.nrs_workspace_size(ctx, pb.N, pb.Q, pb.M, method)
    return torch.empty(nbytes, dtype=torch.uint8, device=DEV)


def gpu_solve(ctx, scene, pb, host, method, **opts):
    ws = workspace(ctx, pb, method)
    sol = torch.empty(pb.n, dtype=torch.float64, device=DEV)
    ft = T(scene["ftext"]) if scene["M"] else None
    info = nrs.nrs_solve(ctx, pb, T(host["u"]), ft, sol, ws, method=method, **opts)
    return sol.cpu().numpy(), info


def rel_force_errors(sol, ref, N):
    """Relative 2-norm errors of the force densities and of (U, Omega)."""
    f, fr = sol[:3 * N], ref[:3 * N]
    ef = np.linalg.norm(f - fr) / np.linalg.norm(fr)
    if len(ref) > 3 * N:
        g, gr = sol[3 * N:], ref[3 * N:]
        eg = np.linalg.norm(g - gr) / max(np.linalg.norm(gr), 1e-300)
    else:
        eg = 0.0
    return ef, eg


def lu_ws(ctx, n, A, bf16=False):
    """Workspace of nrs_lu_factor for an order-n matrix like A."""
    prec = 16 if bf16 else (32 if A.dtype == torch.float32 else 64)
    return torch.empty(nrs.nrs_lu_factor_workspace_size(ctx, n, prec), dtype=torch.uint8,
                       device=DEV)


def lus_ws(ctx, n):
    """Workspace of nrs_lu_solve for order n."""
    return torch.empty(nrs.nrs_lu_solve_workspace_size(ctx, n), dtype=torch.uint8, device=DEV)
