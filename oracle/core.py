"""Plain FP64 reference of the nearest-neighbour regularized stokeslet
(NEAREST) resistance / swimming problem.  Test infrastructure only; see the
package docstring.  Section and equation numbers refer to Gallagher & Smith,
arXiv:2001.06468.

Readings of the paper adopted here (where it is silent or inconsistent):
  * kernels are functions of r = x - y (the regularized formulas are printed
    in terms of "x" alone);
  * the nearest-neighbour form carries a + sign, so f is the force density
    exerted on the fluid by the body;
  * quadrature weights w_q are explicit and the unknown is a force density;
    with all w_q = 1 the operator is the paper's sum over q exactly;
  * unknowns are ordered component-major (f_x[0..N), f_y, f_z) followed by
    (U, Omega) for each free body;
  * rigid-body equations (named but not written in the paper): velocity
    rows  A_s f - U - Omega x r = u_def,  force rows  sum W f = F_ext,
    moment rows  sum W r x f = T_ext,  r = x - x0, W_n = sum_{nu(q)=n} w_q;
  * the nearest-neighbour search is restricted to a group (one body, one
    wall), squared distances in FP64, ties to the lowest index;
  * time stepping is classical RK4 with re-orthonormalisation of the body
    frame after every step.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# kernels (Sec. 2 and Sec. 3)
# ----------------------------------------------------------------------------


def stokeslet_singular(r):
    """Singular stokeslet S_jk = delta_jk/|r| + r_j r_k/|r|^3 (Sec. 2, eq. 5)."""
    r = np.asarray(r, dtype=np.float64)
    d = np.sqrt(np.sum(r * r, axis=-1))
    eye = np.eye(3)
    return (eye / d[..., None, None]
            + r[..., :, None] * r[..., None, :] / (d ** 3)[..., None, None])


def blob(r, eps):
    """Cortez blob phi_eps(r) = 15 eps^4 / (8 pi (|r|^2 + eps^2)^(7/2)) (Sec. 3, eq. 16)."""
    r = np.asarray(r, dtype=np.float64)
    r2 = np.sum(r * r, axis=-1)
    return 15.0 * eps ** 4 / (8.0 * math.pi * (r2 + eps * eps) ** 3.5)


def pressure_reg(r, eps):
    """Regularized pressure P^eps_k = r_k (2|r|^2 + 5 eps^2)/(|r|^2+eps^2)^(5/2)
    (Sec. 3, eq. 17)."""
    r = np.asarray(r, dtype=np.float64)
    r2 = np.sum(r * r, axis=-1)
    return r * ((2.0 * r2 + 5.0 * eps * eps) / (r2 + eps * eps) ** 2.5)[..., None]


def stokeslet_reg(r, eps):
    """Regularized stokeslet
    S^eps_jk = [delta_jk (|r|^2 + 2 eps^2) + r_j r_k] / (|r|^2 + eps^2)^(3/2)
    (Sec. 3, eq. 18), for r of shape (..., 3); returns (..., 3, 3)."""
    r = np.asarray(r, dtype=np.float64)
    r2 = np.sum(r * r, axis=-1)
    num = ((r2 + 2.0 * eps * eps)[..., None, None] * np.eye(3)
           + r[..., :, None] * r[..., None, :])
    return num / ((r2 + eps * eps) ** 1.5)[..., None, None]


# ----------------------------------------------------------------------------
# geometry at time t (Sec. 4: state Y = [X0; B], body-frame shapes)
# ----------------------------------------------------------------------------


def _wave_terms(wave, part, s, t):
    """Body-frame wave displacement, its s-derivative and its t-derivative
    for points whose part index is >= 0 (zeros elsewhere)."""
    n = part.shape[0]
    disp = np.zeros((3, n))
    dds = np.zeros((3, n))
    ddt = np.zeros((3, n))
    sel = part >= 0
    if np.any(sel):
        p = wave[part[sel]]
        beta, A0, A1, k, om, phi = (p[:, i] for i in range(6))
        ss = s[sel]
        th = k * ss - om * t + phi
        amp = A0 + A1 * ss
        disp[0, sel] = beta * ss
        disp[1, sel] = amp * np.sin(th)
        dds[0, sel] = beta
        dds[1, sel] = A1 * np.sin(th) + amp * k * np.cos(th)
        ddt[1, sel] = -om * amp * np.cos(th)
    return disp, dds, ddt, sel


def geometry(scene, t, Y):
    """Lab-frame force points x (3,N), quadrature points X (3,Q), weights w
    (Q,) and prescribed velocities u (3,N) at time t for body states Y
    (M, 12) = [x0 (3), B row-major (9)].

    Free-body points: x = x0 + B xi(t), u = B dxi/dt (deformation velocity).
    Fixed points: x = xi, u = ufix.  Wave quadrature weights scale with the
    arc-length metric |dxi/ds|."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)

    def place(xi, body, part, s):
        disp, dds, ddt, _ = _wave_terms(scene["wave"], part, s, t)
        xi_t = xi + disp
        pos = xi_t.copy()
        vel = np.zeros_like(xi_t)
        for b in range(Y.shape[0]):
            idx = body == b
            if not np.any(idx):
                continue
            x0 = Y[b, :3]
            B = Y[b, 3:].reshape(3, 3)
            pos[:, idx] = x0[:, None] + B @ xi_t[:, idx]
            vel[:, idx] = B @ ddt[:, idx]
        return pos, vel, dds

    x, u, _ = place(scene["xi"], scene["body"], scene["part"], scene["s"])
    fixed = scene["body"] < 0
    u[:, fixed] = scene["ufix"][:, fixed]
    X, _, dds = place(scene["Xi"], scene["bodyX"], scene["partX"], scene["sX"])
    w = scene["w0"].astype(np.float64).copy()
    wav = scene["partX"] >= 0
    w[wav] = w[wav] * np.sqrt(np.sum(dds[:, wav] ** 2, axis=0))
    return x, X, w, u


# ----------------------------------------------------------------------------
# nearest-neighbour map (Sec. 3, eq. 20)
# ----------------------------------------------------------------------------


def nearest(x, X, group_off, groupX):
    """nu[q] = argmin_n |x[n] - X[q]| over the coarse points n of q's group.
    Squared distances are formed as (dx*dx + dy*dy) + dz*dz in FP64; the
    lowest index wins a tie (numpy.argmin returns the first minimum)."""
    Q = X.shape[1]
    nu = np.empty(Q, dtype=np.int32)
    for g in range(len(group_off) - 1):
        lo, hi = int(group_off[g]), int(group_off[g + 1])
        qs = np.nonzero(groupX == g)[0]
        if qs.size == 0:
            continue
        if hi <= lo:
            raise ValueError(f"group {g} has quadrature points but no force points")
        # quadrature points taken in blocks only to bound memory; each q's
        # argmin is computed on its own
        step = max(1, (1 << 24) // (hi - lo))
        for a in range(0, qs.size, step):
            qb = qs[a:a + step]
            dx = x[0, lo:hi][None, :] - X[0, qb][:, None]
            dy = x[1, lo:hi][None, :] - X[1, qb][:, None]
            dz = x[2, lo:hi][None, :] - X[2, qb][:, None]
            d2 = dx * dx + dy * dy + dz * dz
            nu[qb] = lo + np.argmin(d2, axis=1)
    return nu


# ----------------------------------------------------------------------------
# NEAREST operator (Sec. 3, eqs. 21-23 and the matrix view that follows)
# ----------------------------------------------------------------------------


def assemble_As(x, X, w, nu, eps, mu, chunk_pairs=1 << 21):
    """A_s = (8 pi mu)^-1 * S * diag(w (x) 1_3) * nuhat, literally as the
    product of the dense 3N x 3Q stokeslet matrix with the sparse 3Q x 3N
    nearest-neighbour matrix, the Q dimension taken in blocks (Sec. 3,
    matrix view after eq. 23).  Row/column index j*N + m (component-major).
    Within a block only the columns of nuhat that hold an entry of the block
    are formed; every other column of that block's product is zero."""
    N = x.shape[1]
    Q = X.shape[1]
    As = np.zeros((3 * N, 3 * N))
    qc = max(1, chunk_pairs // max(N, 1))
    for q0 in range(0, Q, qc):
        q1 = min(Q, q0 + qc)
        Qc = q1 - q0
        r = (x[:, :, None] - X[:, None, q0:q1]).transpose(1, 2, 0)  # (N, Qc, 3)
        S = stokeslet_reg(r, eps)                                    # (N, Qc, 3, 3)
        # dense block: row j*N + m, column k*Qc + q
        Sd = S.transpose(2, 0, 3, 1).reshape(3 * N, 3 * Qc)
        rows = np.concatenate([k * Qc + np.arange(Qc) for k in range(3)])
        cols = np.concatenate([k * N + nu[q0:q1] for k in range(3)])
        vals = np.concatenate([w[q0:q1]] * 3)
        nuhat = sp.csc_matrix((vals, (rows, cols)), shape=(3 * Qc, 3 * N))
        used = np.unique(cols)
        sub = nuhat[:, used]                       # 3Qc x len(used), sparse
        As[:, used] += (sub.T @ Sd.T).T            # (S diag(w) nuhat)[:, used]
    return As / (8.0 * math.pi * mu)


def patch_weights(w, nu, N):
    """W_n = sum of the quadrature weights of the points whose nearest force
    point is n."""
    return np.bincount(nu, weights=w, minlength=N)[:N]


def assemble_system(As, x, W, body, Y, M):
    """Full swimming-problem matrix (order 3N + 6M) from A_s and the rigid-body
    blocks: velocity rows A_s f - U - Omega x r, force rows sum W f, moment
    rows sum W r x f (Sec. 2 and Sec. 4; equations not printed in the paper)."""
    N = x.shape[1]
    n = 3 * N + 6 * M
    A = np.zeros((n, n))
    A[:3 * N, :3 * N] = As
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)
    e = np.eye(3)
    for m in range(N):
        s = int(body[m])
        if s < 0:
            continue
        r = x[:, m] - Y[s, :3]
        cU = 3 * N + 6 * s
        cO = cU + 3
        for j in range(3):
            A[j * N + m, cU + j] = -1.0
            for i in range(3):
                A[j * N + m, cO + i] = -np.cross(e[i], r)[j]
        for j in range(3):
            A[cU + j, j * N + m] += W[m]
        for i in range(3):
            for k in range(3):
                A[cO + i, k * N + m] += W[m] * np.cross(r, e[k])[i]
    return A


def rhs(u, ftext):
    """b = [u_x; u_y; u_z; (F_ext, T_ext) per body]."""
    return np.concatenate([u.reshape(-1), np.asarray(ftext, dtype=np.float64).reshape(-1)])


def split_solution(sol, N, M):
    return sol[:3 * N].reshape(3, N), sol[3 * N:].reshape(M, 6)


def solve_system(A, b):
    """Dense solve by LAPACK dgesv (LU with partial pivoting)."""
    return np.linalg.solve(A, b)


def condition_1(A):
    """1-norm condition number |A|_1 |A^-1|_1 with the inverse formed
    explicitly (oracle-sized systems)."""
    A = np.asarray(A, dtype=np.float64)
    Ainv = np.linalg.inv(A)
    return float(np.abs(A).sum(axis=0).max() * np.abs(Ainv).sum(axis=0).max())


def solve_with_condition(A, b, overwrite=False):
    """Dense solve by LU with partial pivoting (LAPACK getrf / getrs) and the
    LAPACK 1-norm condition estimate (gecon, Hager's method refined by
    Higham) from the same factors; for systems too large for an explicit
    inverse.  Returns (x, kappa1_estimate).  The estimate never exceeds the
    true kappa_1 and is usually within a factor of a few of it."""
    import scipy.linalg as sla
    from scipy.linalg import lapack
    anorm = float(np.abs(A).sum(axis=0).max())
    lu, piv = sla.lu_factor(A, overwrite_a=overwrite, check_finite=False)
    x = sla.lu_solve((lu, piv), b, check_finite=False)
    gecon = lapack.get_lapack_funcs("gecon", (lu,))
    rcond, info = gecon(lu, anorm, norm="1")
    if info != 0:
        raise RuntimeError(f"gecon info {info}")
    return x, (1.0 / rcond if rcond > 0 else math.inf)


def solve_scene(scene, t=0.0, Y=None, nu=None, return_all=False):
    """Geometry -> nearest map -> A_s -> A -> dgesv for one scene state.
    Returns f (3,N) and UW (M,6) (and a dict of intermediates)."""
    Y = scene["Y0"] if Y is None else Y
    x, X, w, u = geometry(scene, t, Y)
    nu_bf = nearest(x, X, scene["group_off"], scene["groupX"])
    if nu is not None and not np.array_equal(nu, nu_bf):
        raise AssertionError("supplied nearest map differs from brute force")
    N, M = scene["N"], scene["M"]
    As = assemble_As(x, X, w, nu_bf, scene["eps"], scene["mu"])
    W = patch_weights(w, nu_bf, N)
    A = assemble_system(As, x, W, scene["body"], Y, M)
    b = rhs(u, scene["ftext"])
    sol = solve_system(A, b)
    f, UW = split_solution(sol, N, M)
    if return_all:
        return f, UW, dict(x=x, X=X, w=w, u=u, nu=nu_bf, As=As, W=W, A=A, b=b, sol=sol)
    return f, UW


# ----------------------------------------------------------------------------
# textbook LU (cross-check of the LAPACK solve on small systems)
# ----------------------------------------------------------------------------


def doolittle_solve(A, b):
    """Gaussian elimination with partial pivoting in pure Python loops
    (first maximal |pivot|, lowest row on ties), then substitution."""
    n = len(b)
    a = [list(map(float, row)) for row in np.asarray(A)]
    y = list(map(float, b))
    for k in range(n):
        p = k
        best = abs(a[k][k])
        for i in range(k + 1, n):
            if abs(a[i][k]) > best:
                best, p = abs(a[i][k]), i
        if best == 0.0:
            raise ZeroDivisionError("singular matrix")
        if p != k:
            a[k], a[p] = a[p], a[k]
            y[k], y[p] = y[p], y[k]
        piv = a[k][k]
        rowk = a[k]
        for i in range(k + 1, n):
            l = a[i][k] / piv
            if l != 0.0:
                rowi = a[i]
                rowi[k] = l
                for j in range(k + 1, n):
                    rowi[j] -= l * rowk[j]
                y[i] -= l * y[k]
    xs = [0.0] * n
    for i in range(n - 1, -1, -1):
        s = y[i]
        for j in range(i + 1, n):
            s -= a[i][j] * xs[j]
        xs[i] = s / a[i][i]
    return np.array(xs)


# ----------------------------------------------------------------------------
# time stepping (Sec. 4: Y' = F(Y, t))
# ----------------------------------------------------------------------------


def rates(Y, UW):
    """dx0/dt = U, dB/dt = [Omega]x B (each body axis rotates with Omega)."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)
    dY = np.zeros_like(Y)
    for b in range(Y.shape[0]):
        U = UW[b, :3]
        Om = UW[b, 3:]
        B = Y[b, 3:].reshape(3, 3)
        dB = np.cross(Om[None, :], B.T).T
        dY[b, :3] = U
        dY[b, 3:] = dB.ravel()
    return dY


def orthonormalise(Y):
    """Modified Gram-Schmidt on the three columns of each body frame."""
    Y = np.array(Y, dtype=np.float64).reshape(-1, 12)
    for b in range(Y.shape[0]):
        B = Y[b, 3:].reshape(3, 3).copy()
        q0 = B[:, 0] / np.linalg.norm(B[:, 0])
        v1 = B[:, 1] - (q0 @ B[:, 1]) * q0
        q1 = v1 / np.linalg.norm(v1)
        v2 = B[:, 2] - (q0 @ B[:, 2]) * q0
        v2 = v2 - (q1 @ v2) * q1
        q2 = v2 / np.linalg.norm(v2)
        Y[b, 3:] = np.stack([q0, q1, q2], axis=1).ravel()
    return Y


def rk4_generic(F, y, t, dt):
    """Classical fourth-order Runge-Kutta step for y' = F(y, t)."""
    k1 = F(y, t)
    k2 = F(y + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = F(y + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = F(y + dt * k3, t + dt)
    return y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4_step(scene, Y, t, dt):
    """One RK4 step of the swimmer state; each stage recomputes the geometry,
    the nearest map and the full solve, then the frames are re-orthonormalised."""
    M = scene["M"]

    def F(y, tt):
        _, UW = solve_scene(scene, tt, y.reshape(M, 12))
        return rates(y.reshape(M, 12), UW)

    Yn = rk4_generic(F, np.asarray(Y, dtype=np.float64).reshape(M, 12), t, dt)
    return orthonormalise(Yn)


# ----------------------------------------------------------------------------
# restarted GMRES (Saad & Schultz), used for the learned warm-start checks
# ----------------------------------------------------------------------------


def gmres(A, b, x0=None, tol=1e-8, restart=50, maxit=1000):
    """Restarted GMRES(m) with modified Gram-Schmidt Arnoldi and Givens
    rotations; stops when ||b - A x|| <= tol * ||b||.  Returns (x, iters,
    relres)."""
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0, 0.0
    it = 0
    r = b - A @ x
    beta = np.linalg.norm(r)
    while beta > tol * bn and it < maxit:
        m = restart
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_used = 0
        for k in range(m):
            wv = A @ V[:, k]
            for i in range(k + 1):
                H[i, k] = V[:, i] @ wv
                wv = wv - H[i, k] * V[:, i]
            H[k + 1, k] = np.linalg.norm(wv)
            if H[k + 1, k] != 0.0:
                V[:, k + 1] = wv / H[k + 1, k]
            for i in range(k):
                tmp = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = tmp
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_used = k + 1
            if abs(g[k + 1]) <= tol * bn or it >= maxit:
                break
        yk = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + V[:, :k_used] @ yk
        r = b - A @ x
        beta = np.linalg.norm(r)
    return x, it, beta / bn
