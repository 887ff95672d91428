"""Pins of the oracle's nearest map, NEAREST operator and rigid-body system
(Sec. 3 eqs. 20-23, Sec. 4) against brute force, special cases and exact
invariants."""
import math

import numpy as np
import pytest

import oracle
import synth


def _random_cloud(rng, N, Q, G=2):
    x = rng.normal(size=(3, N))
    X = rng.normal(size=(3, Q))
    sizes = np.full(G, N // G)
    sizes[-1] += N - sizes.sum()
    go = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    gX = rng.integers(0, G, size=Q).astype(np.int32)
    return x, X, go, gX


def test_nearest_matches_pure_python_brute_force():
    rng = np.random.default_rng(0)
    x, X, go, gX = _random_cloud(rng, 13, 71, G=3)
    nu = oracle.nearest(x, X, go, gX)
    for q in range(X.shape[1]):
        g = gX[q]
        best, arg = None, None
        for n in range(go[g], go[g + 1]):
            d = math.dist(x[:, n], X[:, q])
            if best is None or d < best:
                best, arg = d, n
        assert nu[q] == arg


def test_nearest_tie_goes_to_lowest_index():
    x = np.array([[1.0, -1.0, 1.0], [0, 0, 0], [0, 0, 0]])
    X = np.zeros((3, 1))
    nu = oracle.nearest(x, X, np.array([0, 3], np.int32), np.zeros(1, np.int32))
    assert nu[0] == 0
    nu = oracle.nearest(x[:, ::-1].copy(), X, np.array([0, 3], np.int32), np.zeros(1, np.int32))
    assert nu[0] == 0


def _entrywise_As(x, X, w, nu, eps, mu):
    """Sec. 3 eq. 23 term by term in pure Python loops."""
    N, Q = x.shape[1], X.shape[1]
    A = [[0.0] * (3 * N) for _ in range(3 * N)]
    for m in range(N):
        for q in range(Q):
            r = [x[i, m] - X[i, q] for i in range(3)]
            r2 = r[0] ** 2 + r[1] ** 2 + r[2] ** 2
            den = (r2 + eps * eps) ** 1.5
            n = nu[q]
            for j in range(3):
                for k in range(3):
                    s = ((r2 + 2 * eps * eps) if j == k else 0.0) + r[j] * r[k]
                    A[j * N + m][k * N + n] += w[q] * s / den / (8 * math.pi * mu)
    return np.array(A)


def test_operator_matches_entrywise_sum():
    rng = np.random.default_rng(1)
    x, X, go, gX = _random_cloud(rng, 7, 53, G=2)
    w = rng.random(53) + 0.5
    nu = oracle.nearest(x, X, go, gX)
    A = oracle.assemble_As(x, X, w, nu, 0.2, 1.3, chunk_pairs=20)  # several Q blocks
    B = _entrywise_As(x, X, w, nu, 0.2, 1.3)
    assert np.max(np.abs(A - B)) <= 1e-14 * np.max(np.abs(B))


def test_nystrom_special_case_is_symmetric_kernel_matrix():
    """Q = N, X = x, nu = identity, w = 1: A_s is the Nystrom matrix of
    Sec. 3 eq. 13 (without its sign), exactly symmetric."""
    rng = np.random.default_rng(2)
    N = 9
    x = rng.normal(size=(3, N))
    A = oracle.assemble_As(x, x.copy(), np.ones(N), np.arange(N, dtype=np.int32), 0.1, 1.0)
    np.testing.assert_array_equal(A, A.T)
    for m in range(N):
        for n in range(N):
            blk = A[m::N, n::N]
            ref = oracle.stokeslet_reg(x[:, m] - x[:, n], 0.1) / (8 * math.pi)
            np.testing.assert_allclose(blk, ref, rtol=1e-14, atol=0)


def test_uniform_filament_gives_symmetric_operator():
    """Straight uniform filament with parent-cell nearest map: congruent cells
    with sub-points symmetric about their centre make A_s symmetric."""
    N, sub = 12, 8
    s = (np.arange(N) + 0.5) / N
    sq = (np.arange(N * sub) + 0.5) / (N * sub)
    x = np.stack([s, 0 * s, 0 * s])
    X = np.stack([sq, 0 * sq, 0 * sq])
    nu = oracle.nearest(x, X, np.array([0, N], np.int32), np.zeros(N * sub, np.int32))
    np.testing.assert_array_equal(nu, np.repeat(np.arange(N), sub))
    A = oracle.assemble_As(x, X, np.full(N * sub, 1.0 / (N * sub)), nu, 0.01, 1.0)
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))


def test_rotation_translation_permutation_covariance():
    rng = np.random.default_rng(4)
    x, X, go, gX = _random_cloud(rng, 8, 40, G=1)
    w = rng.random(40)
    nu = oracle.nearest(x, X, go, gX)
    A = oracle.assemble_As(x, X, w, nu, 0.15, 1.0)
    N = 8
    R = synth.random_rotation(rng)
    Ar = oracle.assemble_As(R @ x, R @ X, w, nu, 0.15, 1.0)
    for m in range(N):
        for n in range(N):
            np.testing.assert_allclose(Ar[m::N, n::N], R @ A[m::N, n::N] @ R.T,
                                       atol=1e-13 * np.abs(A).max())
    t = rng.normal(size=(3, 1))
    At = oracle.assemble_As(x + t, X + t, w, nu, 0.15, 1.0)
    np.testing.assert_allclose(At, A, atol=1e-13 * np.abs(A).max())
    p = rng.permutation(N)
    inv = np.argsort(p)
    Ap = oracle.assemble_As(x[:, p], X, w, inv[nu].astype(np.int32), 0.15, 1.0)
    idx = np.concatenate([k * N + p for k in range(3)])
    np.testing.assert_allclose(Ap, A[np.ix_(idx, idx)], atol=1e-14 * np.abs(A).max())


def _swimmer_like():
    return synth.filament_scene(M=2, seed=5, Nf=10, Qf=60)


def test_rigid_motion_gives_zero_force_exactly():
    """u_m = V + W x r_m on every free-body point: f = 0, U = -V, Omega = -W
    solves the system exactly (K columns of the rigid-body block)."""
    sc = _swimmer_like()
    Y = sc["Y0"]
    x, X, w, _ = oracle.geometry(sc, 0.3, Y)
    nu = oracle.nearest(x, X, sc["group_off"], sc["groupX"])
    As = oracle.assemble_As(x, X, w, nu, sc["eps"], sc["mu"])
    W = oracle.patch_weights(w, nu, sc["N"])
    A = oracle.assemble_system(As, x, W, sc["body"], Y, sc["M"])
    V = np.array([[0.3, -0.2, 0.5], [-1.0, 0.1, 0.2]])
    Wr = np.array([[0.0, 0.7, -0.4], [0.2, 0.2, 0.9]])
    u = np.zeros((3, sc["N"]))
    for m in range(sc["N"]):
        b = sc["body"][m]
        u[:, m] = V[b] + np.cross(Wr[b], x[:, m] - Y[b, :3])
    sol = oracle.solve_system(A, oracle.rhs(u, np.zeros((2, 6))))
    f, UW = oracle.split_solution(sol, sc["N"], sc["M"])
    scale = np.abs(UW).max()
    assert np.abs(f).max() < 1e-10 * scale / np.abs(As).max()
    np.testing.assert_allclose(UW[:, :3], -V, atol=1e-12)
    np.testing.assert_allclose(UW[:, 3:], -Wr, atol=1e-12)


def test_resistance_and_mobility_forms_agree():
    """Resistance solve of a sphere moving rigidly gives forces f_R; the
    mobility solve driven by the resulting total force and moment returns
    the same motion and the same f (B rows against K columns)."""
    V = np.array([0.4, -0.1, 0.25])
    Om = np.array([0.1, 0.3, -0.2])
    res = synth.sphere_scene(4, 12, U=V, Omega=Om)
    f_R, _, d = oracle.solve_scene(res, return_all=True)
    F = (d["W"][None, :] * f_R).sum(axis=1)
    T = (d["W"][None, :] * np.cross(d["x"].T, f_R.T).T).sum(axis=1)
    mob = synth.sphere_scene(4, 12, free=True, force=F, torque=T)
    f_M, UW = oracle.solve_scene(mob)
    np.testing.assert_allclose(UW[0, :3], V, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(UW[0, 3:], Om, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(f_M, f_R, atol=1e-9 * np.abs(f_R).max())


def test_lapack_solve_matches_textbook_elimination():
    sc = synth.sphere_scene(3, 9)
    _, _, d = oracle.solve_scene(sc, return_all=True)
    x_ref = oracle.doolittle_solve(d["A"], d["b"])
    np.testing.assert_allclose(d["sol"], x_ref, rtol=1e-11, atol=1e-13)
    r = d["b"] - d["A"] @ d["sol"]
    n = len(d["b"])
    bw = np.abs(r).max() / (np.abs(d["A"]).sum(1).max() * np.abs(d["sol"]).max() + np.abs(d["b"]).max())
    assert bw <= 10 * n * 2.0 ** -53


def _kappa1_by_columns(A):
    """kappa_1 = |A|_1 |A^-1|_1 with the columns of A^-1 found one by one by
    the textbook elimination (pure Python)."""
    n = A.shape[0]
    cols = [oracle.doolittle_solve(A, np.eye(n)[:, j]) for j in range(n)]
    norm_inv = max(sum(abs(v) for v in c) for c in cols)
    norm_a = max(sum(abs(A[i, j]) for i in range(n)) for j in range(n))
    return norm_a * norm_inv


def test_condition_1_closed_forms():
    """Diagonal matrix: max |d| / min |d|.  Hilbert matrix of order 4: the
    textbook value 28375 (|H|_1 = 25/12, |H^-1|_1 = 13620)."""
    d = np.array([3.0, -0.5, 8.0, 0.25])
    assert oracle.condition_1(np.diag(d)) == pytest.approx(32.0, rel=1e-14)
    H = np.array([[1.0 / (i + j + 1) for j in range(4)] for i in range(4)])
    assert oracle.condition_1(H) == pytest.approx(28375.0, rel=1e-9)
    rng = np.random.default_rng(4)
    A = rng.normal(size=(7, 7))
    assert oracle.condition_1(A) == pytest.approx(_kappa1_by_columns(A), rel=1e-10)


def test_solve_with_condition_against_textbook_elimination():
    """The getrf/getrs solve equals the textbook elimination, and the gecon
    estimate is a lower bound of the exact kappa_1 within a factor 3 (on the
    sphere system, a random matrix and the Hilbert matrix of order 6)."""
    sc = synth.sphere_scene(3, 9)
    _, _, d = oracle.solve_scene(sc, return_all=True)
    x, kap = oracle.solve_with_condition(d["A"], d["b"])
    np.testing.assert_allclose(x, oracle.doolittle_solve(d["A"], d["b"]), rtol=1e-11, atol=1e-13)
    rng = np.random.default_rng(5)
    H6 = np.array([[1.0 / (i + j + 1) for j in range(6)] for i in range(6)])
    for A in (d["A"], rng.normal(size=(40, 40)), H6):
        b = np.ones(A.shape[0])
        x, kap = oracle.solve_with_condition(A, b)
        exact = oracle.condition_1(A)
        assert exact / 3.0 <= kap <= exact * (1 + 1e-8), (kap, exact)
        np.testing.assert_allclose(A @ x, b, atol=1e-9 * exact * np.abs(b).max())
    # overwrite=True leaves the result unchanged
    A = rng.normal(size=(30, 30))
    b = rng.normal(size=30)
    x1, k1 = oracle.solve_with_condition(A, b)
    x2, k2 = oracle.solve_with_condition(A.copy(order="F"), b, overwrite=True)
    np.testing.assert_array_equal(x1, x2)
    assert k1 == k2
