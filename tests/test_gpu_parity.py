"""Parity of every C-ABI entry point with the CPU FP64 oracle on the same
seeded inputs (MI355X).  Tolerances:
  geometry, FP64 assembly, FP64 apply : 1e-13 relative to the largest entry
    (different summation order only);
  FP32 assembly : 4e-6 of the largest entry (about 30 FP32 ulps: a 16-term
    segment sum of products with a hardware reciprocal square root);
  nearest map : bit-exact (integer);
  solves : relative 2-norm error of forces and of (U, Omega) <= 1e-8, the
    target stated for the refined forms.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2001_06468_amd as nrs
    from gpu_util import (T, prepare, oracle_system, workspace, gpu_solve, rel_force_errors, DEV,
                          lu_ws, lus_ws)


@pytest.fixture(scope="module")
def ctx():
    c = nrs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _scenes_small():
    return [
        ("sphere_nc4_nq16", synth.sphere_scene(4, 16)),
        ("filaments_M5", synth.filament_scene(5, seed=0)),
        ("sperm_K2_h8", synth.sperm_channel_scene(2, h=1.0 / 8, seed=1, Nh=30, Qh=300)),
        ("rodwall_700", synth.rod_wall_batch(1, seed=3, lo=700, hi=700)[0]),
        ("sphere_free", synth.sphere_scene(3, 9, free=True, force=np.array([0, 0, -1.0]))),
    ]


SCENES = _scenes_small()


def test_library_version():
    assert nrs.nrs_version().startswith("nrs ")


@pytest.mark.parametrize("name,scene", SCENES, ids=[s[0] for s in SCENES])
def test_geometry(ctx, name, scene):
    rng = np.random.default_rng(7)
    Y = scene["Y0"].copy()
    if scene["M"]:
        Y[:, :3] += 0.01 * rng.normal(size=(scene["M"], 3))
    t = 0.83
    x, X, w, u = oracle.geometry(scene, t, Y)
    ds = nrs.DeviceScene(scene)
    gx = torch.empty(3 * scene["N"], dtype=torch.float64, device=DEV)
    gX = torch.empty(3 * scene["Q"], dtype=torch.float64, device=DEV)
    gw = torch.empty(scene["Q"], dtype=torch.float64, device=DEV)
    gu = torch.empty(3 * scene["N"], dtype=torch.float64, device=DEV)
    nrs.nrs_geometry(ctx, ds, t, T(Y) if scene["M"] else None, gx, gX, gw, gu)
    for g, r in ((gx, x), (gX, X), (gw, w), (gu, u)):
        g = g.cpu().numpy().reshape(r.shape)
        assert np.max(np.abs(g - r)) <= 1e-13 * max(1.0, np.max(np.abs(r)))


@pytest.mark.parametrize("name,scene", SCENES, ids=[s[0] for s in SCENES])
def test_nearest_bit_exact(ctx, name, scene):
    x, X, _, _ = oracle.geometry(scene, 0.4, scene["Y0"])
    ref = oracle.nearest(x, X, scene["group_off"], scene["groupX"])
    nu = torch.empty(scene["Q"], dtype=torch.int32, device=DEV)
    nrs.nrs_nearest(ctx, T(x), scene["group_off"], T(X), T(scene["groupX"], torch.int32), nu)
    np.testing.assert_array_equal(nu.cpu().numpy(), ref)


def test_nearest_ties_and_ragged(ctx):
    """Exact ties resolve to the lowest index; several groups; Q not a
    multiple of the block size."""
    x = np.array([[1.0, -1.0, 0.0, 5.0, 5.0], [0, 0, 1.0, 0, 0], [0, 0, 0, 1.0, -1.0]])
    X = np.zeros((3, 301))
    X[0, 200:] = 5.0
    gX = np.zeros(301, np.int32)
    gX[200:] = 1
    go = np.array([0, 3, 5], np.int32)
    ref = oracle.nearest(x, X, go, gX)
    assert ref[0] == 0 and ref[250] == 3
    nu = torch.empty(301, dtype=torch.int32, device=DEV)
    nrs.nrs_nearest(ctx, T(x), go, T(X), T(gX, torch.int32), nu)
    np.testing.assert_array_equal(nu.cpu().numpy(), ref)


@pytest.mark.parametrize("name,scene", SCENES, ids=[s[0] for s in SCENES])
@pytest.mark.parametrize("precision", [64, 32])
def test_assemble(ctx, name, scene, precision):
    pb, host = prepare(scene, 0.2)
    A_ref, _ = oracle_system(scene, host)
    n = pb.n
    lda = nrs.lda_for(n) + 3
    dt = torch.float64 if precision == 64 else torch.float32
    A = torch.full((n, lda), float("nan"), dtype=dt, device=DEV)  # column-major: row = column
    ws = workspace(ctx, pb, nrs.NRS_FP64_LU if precision == 64 else nrs.NRS_FP32_IR)
    nrs.nrs_assemble(ctx, pb, precision, A, lda, ws)
    G = A.cpu().numpy().astype(np.float64)[:, :n].T
    assert np.all(np.isfinite(G))
    scale = np.max(np.abs(A_ref))
    err = np.max(np.abs(G - A_ref)) / scale
    assert err <= (1e-13 if precision == 64 else 4e-6), err


@pytest.mark.parametrize("name,scene", SCENES, ids=[s[0] for s in SCENES])
def test_apply_fp64(ctx, name, scene):
    pb, host = prepare(scene, 0.9)
    A_ref, _ = oracle_system(scene, host)
    v = np.random.default_rng(2).normal(size=pb.n)
    y = torch.empty(pb.n, dtype=torch.float64, device=DEV)
    nrs.nrs_apply(ctx, pb, T(v), y, workspace(ctx, pb, nrs.NRS_FP64_LU))
    ref = A_ref @ v
    scale = np.max(np.abs(A_ref) @ np.abs(v))
    assert np.max(np.abs(y.cpu().numpy() - ref)) <= 1e-13 * scale


def test_assemble_and_apply_skip_out_of_range_nu(ctx):
    """Quadrature points whose nu is outside [0, N) contribute nothing: the
    FP64 assembly and the matrix-free product equal the oracle's system of
    the same scene with those points removed."""
    name, scene = SCENES[0]
    pb, host = prepare(scene, 0.3)
    N, Q = scene["N"], scene["Q"]
    nu = host["nu"].copy()
    bad = np.array([0, Q // 3, Q - 1])
    nu[bad] = [-1, N, N + 7]
    keep = np.setdiff1d(np.arange(Q), bad)
    trimmed = dict(host, X=host["X"][:, keep], w=host["w"][keep], nu=host["nu"][keep])
    A_ref, _ = oracle_system(scene, trimmed)
    pbad = nrs.Problem(T(host["x"]), T(host["X"]), T(host["w"]), T(nu, torch.int32),
                       T(scene["body"], torch.int32), T(host["Y"]) if scene["M"] else None,
                       scene["eps"], scene["mu"])
    n = pb.n
    lda = nrs.lda_for(n)
    A = torch.full((n, lda), float("nan"), dtype=torch.float64, device=DEV)
    nrs.nrs_assemble(ctx, pbad, 64, A, lda, workspace(ctx, pbad, nrs.NRS_FP64_LU))
    G = A.cpu().numpy()[:, :n].T
    assert np.max(np.abs(G - A_ref)) <= 1e-13 * np.max(np.abs(A_ref))
    v = np.random.default_rng(5).normal(size=n)
    y = torch.empty(n, dtype=torch.float64, device=DEV)
    nrs.nrs_apply(ctx, pbad, T(v), y, workspace(ctx, pbad, nrs.NRS_FP64_LU))
    assert np.max(np.abs(y.cpu().numpy() - A_ref @ v)) <= 1e-13 * np.max(np.abs(A_ref) @ np.abs(v))


def _lu_check(A0, LU, perm, scope, nb=64, tol=1e-12):
    """scope 0: A0[perm] = L U.  scope 1 (static block pivoting): A0 = Lt U,
    where Lt is L with the rows of each diagonal tile L_mm put back at their
    original positions perm[64m + r] (tiles left of the diagonal keep the
    original row order)."""
    n = A0.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    if scope == 0:
        err = np.max(np.abs(A0[perm] - L @ U)) / np.max(np.abs(A0))
        assert np.max(np.abs(np.tril(LU, -1))) <= 1.0 + 1e-12
    else:
        Lt = L.copy()
        for k in range(0, n, nb):
            e = min(n, k + nb)
            assert sorted(perm[k:e]) == list(range(k, e))
            Lt[perm[k:e], k:e] = L[k:e, k:e]
            blk = LU[k:e, k:e]
            assert np.max(np.abs(np.tril(blk, -1)), initial=0.0) <= 1.0 + 1e-6
        err = np.max(np.abs(A0 - Lt @ U)) / np.max(np.abs(A0))
    assert err <= tol * n, err


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 130, 300, 515])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("scope", [0, 1])
def test_lu_factor_and_solve(ctx, n, precision, scope):
    rng = np.random.default_rng(n)
    A0 = rng.normal(size=(n, n)) + (n ** 0.5) * np.eye(n) * (scope == 1)
    dt = torch.float64 if precision == 64 else torch.float32
    lda = nrs.lda_for(n) + 5
    A = torch.zeros((n, lda), dtype=dt, device=DEV)
    A[:, :n] = torch.from_numpy(A0.T.copy()).to(dt)
    ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    sing = torch.zeros(1, dtype=torch.int32, device=DEV)
    nrs.nrs_lu_factor(ctx, A, lda, ipiv, perm, sing, lu_ws(ctx, n, A), pivot_scope=scope)
    LU = A.cpu().numpy().astype(np.float64)[:, :n].T
    p = perm.cpu().numpy()
    piv = ipiv.cpu().numpy()
    # the permutation is the composition of the LAPACK-style interchanges
    q = np.arange(n)
    for j in range(n):
        q[[j, piv[j]]] = q[[piv[j], j]]
    np.testing.assert_array_equal(p, q)
    assert sing.item() == 0
    A0c = A0.astype(np.float32).astype(np.float64) if precision == 32 else A0
    _lu_check(A0c, LU, p, scope, tol=1e-13 if precision == 64 else 3e-6)
    b = rng.normal(size=n)
    xs = torch.empty(n, dtype=dt, device=DEV)
    nrs.nrs_lu_solve(ctx, A, lda, perm, T(b, dt), xs, lus_ws(ctx, n), pivot_scope=scope)
    ref = np.linalg.solve(A0c, b)
    err = np.linalg.norm(xs.cpu().numpy() - ref) / np.linalg.norm(ref)
    unit = 2.0 ** -53 if precision == 64 else 2.0 ** -24
    assert err <= 10 * n * unit * np.linalg.cond(A0c), err


@pytest.mark.parametrize("scope", [0, 1])
def test_lu_singular_flag(ctx, scope):
    n = 70
    A0 = np.random.default_rng(0).normal(size=(n, n))
    A0[:, 5] = 0.0
    A = torch.from_numpy(A0.T.copy()).to(DEV)
    ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    sing = torch.zeros(1, dtype=torch.int32, device=DEV)
    nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, lu_ws(ctx, n, A), pivot_scope=scope)
    assert sing.item() == 1


def _pow2_scale(v):
    """2^-floor(log2 v) for v > 0, else 1 (FP32 values)."""
    out = np.ones_like(v)
    pos = v > 0
    out[pos] = np.ldexp(np.float32(1.0), -np.floor(np.log2(v[pos].astype(np.float64))).astype(int))
    return out.astype(np.float32)


@pytest.mark.parametrize("n", [1, 65, 300])
def test_equilibrate_matches_definition(ctx, n):
    """nrs_equilibrate against its definition computed here in NumPy: the
    power-of-two row factors from the row maxima, the column factors from the
    maxima of the row-scaled columns, and the scaled matrix, all bit for bit
    (powers of two scale exactly); an all-zero row and column keep factor 1;
    every row and column maximum of the result is in [1, 2)."""
    rng = np.random.default_rng(n)
    A0 = (rng.normal(size=(n, n)) * np.exp(rng.uniform(-20, 20, size=(n, 1)))
          * np.exp(rng.uniform(-20, 20, size=(1, n)))).astype(np.float32)
    if n > 2:
        A0[1, :] = 0.0
        A0[:, 2] = 0.0
    lda = nrs.lda_for(n) + 3
    A = torch.zeros((n, lda), dtype=torch.float32, device=DEV)
    A[:, :n] = torch.from_numpy(A0.T.copy()).to(DEV)
    dr = torch.empty(n, dtype=torch.float32, device=DEV)
    dc = torch.empty(n, dtype=torch.float32, device=DEV)
    ws = torch.empty(4 * n, dtype=torch.uint8, device=DEV)
    nrs.nrs_equilibrate(ctx, A, lda, dr, dc, ws)
    r_ref = _pow2_scale(np.abs(A0).max(axis=1))
    c_ref = _pow2_scale((np.abs(A0) * r_ref[:, None]).max(axis=0))
    np.testing.assert_array_equal(dr.cpu().numpy(), r_ref)
    np.testing.assert_array_equal(dc.cpu().numpy(), c_ref)
    S = A.cpu().numpy()[:, :n].T
    np.testing.assert_array_equal(S, A0 * r_ref[:, None] * c_ref[None, :])
    rows, cols = np.abs(S).max(axis=1), np.abs(S).max(axis=0)
    nz_r, nz_c = rows > 0, cols > 0
    assert np.all(cols[nz_c] >= 1) and np.all(cols[nz_c] < 2)
    assert np.all(rows[nz_r] < 2)
    if n > 2:
        assert dr[1].item() == 1.0 and dc[2].item() == 1.0


def test_lu_timeout_word_cleared_each_call(ctx):
    """The factor and solve workspaces carry the wait-timeout word of their
    last call: a word left set (here planted from the host) is cleared by the
    next call, which then runs to the correct result, and nrs_lu_query
    reports 0."""
    n = 300
    rng = np.random.default_rng(3)
    A0 = rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)
    b = rng.normal(size=n)
    A = torch.from_numpy(A0.T.copy()).to(torch.float32).to(DEV)
    ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    sing = torch.zeros(1, dtype=torch.int32, device=DEV)
    wf, wsv = lu_ws(ctx, n, A), lus_ws(ctx, n)
    for ws in (wf, wsv):
        head = (-ws.data_ptr()) % 256          # the head starts at the first 256-byte boundary
        ws[head + 8:head + 12].view(torch.int32).fill_(1)
        assert nrs.nrs_lu_query(ctx, ws) == 1
    nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, wf, pivot_scope=1)
    assert nrs.nrs_lu_query(ctx, wf) == 0
    xs = torch.empty(n, dtype=torch.float32, device=DEV)
    nrs.nrs_lu_solve(ctx, A, n, perm, T(b, torch.float32), xs, wsv, pivot_scope=1)
    assert nrs.nrs_lu_query(ctx, wsv) == 0
    ref = np.linalg.solve(A0, b)
    assert np.linalg.norm(xs.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-4
    with pytest.raises(nrs.NrsError, match="workspace"):
        nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, wf[:64], pivot_scope=1)
    with pytest.raises(nrs.NrsError, match="workspace"):
        nrs.nrs_lu_solve(ctx, A, n, perm, T(b, torch.float32), xs, wsv[:64], pivot_scope=1)


def test_lu_tiles_repeatable_and_large(ctx):
    """The tile LU clears its own flags: back-to-back factorisations of
    different sizes give identical results to fresh ones; n = 3150 spans 50
    tiles with a ragged last tile."""
    rng = np.random.default_rng(11)
    for n in (3150, 200, 3150):
        A0 = rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)
        A = torch.from_numpy(A0.T.copy()).to(torch.float32).to(DEV)
        ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
        perm = torch.empty(n, dtype=torch.int32, device=DEV)
        sing = torch.zeros(1, dtype=torch.int32, device=DEV)
        nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, lu_ws(ctx, n, A), pivot_scope=1)
        b = rng.normal(size=n)
        xs = torch.empty(n, dtype=torch.float32, device=DEV)
        nrs.nrs_lu_solve(ctx, A, n, perm, T(b, torch.float32), xs, lus_ws(ctx, n), pivot_scope=1)
        ref = np.linalg.solve(A0, b)
        err = np.linalg.norm(xs.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err < 1e-4, (n, err)


def test_lu_tiles_bf16_updates(ctx):
    """Tile LU whose trailing updates take BF16 copies of the tiles (FP32
    accumulation): a usable preconditioner (solve error at the level of BF16
    rounding, above the FP32 factorisation's), repeatable bit for bit, and the
    flags clear between sizes (ragged last tile at 3150 and 1000)."""
    rng = np.random.default_rng(12)
    for n in (3150, 200, 1000):
        A0 = rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)
        b = rng.normal(size=n)
        ref = np.linalg.solve(A0, b)
        errs, outs = [], []
        for bf in (True, True, False):
            A = torch.from_numpy(A0.T.copy()).to(torch.float32).to(DEV)
            ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
            perm = torch.empty(n, dtype=torch.int32, device=DEV)
            sing = torch.zeros(1, dtype=torch.int32, device=DEV)
            nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, lu_ws(ctx, n, A, bf), pivot_scope=1,
                              bf16_updates=bf)
            xs = torch.empty(n, dtype=torch.float32, device=DEV)
            nrs.nrs_lu_solve(ctx, A, n, perm, T(b, torch.float32), xs, lus_ws(ctx, n), pivot_scope=1)
            x = xs.cpu().numpy()
            outs.append(A.cpu().numpy())
            errs.append(np.linalg.norm(x - ref) / np.linalg.norm(ref))
        assert np.array_equal(outs[0], outs[1]), n
        assert errs[0] < 2e-2 and errs[2] < 1e-4, (n, errs)
        assert errs[2] < errs[0], (n, errs)


def test_lu_tiles_repeatable(ctx):
    """Repeated single-system tile-LU factorisations of the same matrix are
    bit-identical (every tile's stores land before its completion flag), in
    FP32 and with BF16 update inputs, for a ragged and a tile-aligned order."""
    rng = np.random.default_rng(21)
    for n in (3150, 1024):
        A0 = torch.from_numpy((rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)).T.copy())
        A0 = A0.to(torch.float32).to(DEV)
        for bf in (False, True):
            first = None
            for rep in range(10):
                A = A0.clone()
                ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
                perm = torch.empty(n, dtype=torch.int32, device=DEV)
                sing = torch.zeros(1, dtype=torch.int32, device=DEV)
                nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, lu_ws(ctx, n, A, bf), pivot_scope=1,
                              bf16_updates=bf)
                if first is None:
                    first = (A, perm)
                    continue
                assert torch.equal(A, first[0]) and torch.equal(perm, first[1]), (n, bf, rep)



@pytest.mark.parametrize("n", [5120, 5184])
def test_lu_tiles_row_handover_boundary(ctx, n):
    """Single FP32 systems of up to 80 tile rows hand each diagonal task the
    preceding row tile to solve itself; n = 5120 (80 tile rows) takes that
    path, n = 5184 (81) the plain one.  Both factor P A = L U to FP32
    accuracy, and repeated calls are bit-identical."""
    rng = np.random.default_rng(n)
    A0 = rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)
    lda = nrs.lda_for(n)
    Ad = torch.zeros((n, lda), dtype=torch.float32)
    Ad[:, :n] = torch.from_numpy(A0.T.copy()).to(torch.float32)
    Ad = Ad.to(DEV)
    outs = []
    for rep in range(2):
        A = Ad.clone()
        ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
        perm = torch.empty(n, dtype=torch.int32, device=DEV)
        sing = torch.zeros(1, dtype=torch.int32, device=DEV)
        nrs.nrs_lu_factor(ctx, A, lda, ipiv, perm, sing, lu_ws(ctx, n, A), pivot_scope=1)
        assert sing.item() == 0
        outs.append((A.cpu(), perm.cpu()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    LU = outs[0][0].numpy().astype(np.float64)[:, :n].T
    A0c = A0.astype(np.float32).astype(np.float64)
    _lu_check(A0c, LU, outs[0][1].numpy(), 1, tol=3e-6)

SOLVE_CASES = [
    ("sphere_c1", lambda: synth.sphere_scene(4, 16)),
    ("filaments_M1", lambda: synth.filament_scene(1, seed=0)),
    ("filaments_M5", lambda: synth.filament_scene(5, seed=1)),
    ("sperm_K2_h8", lambda: synth.sperm_channel_scene(2, h=1.0 / 8, seed=1, Nh=30, Qh=300)),
    ("rodwall_700", lambda: synth.rod_wall_batch(1, seed=3, lo=700, hi=700)[0]),
]


@pytest.mark.parametrize("name,mk", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
@pytest.mark.parametrize("method", ["FP64_LU", "FP32_IR", "FP32_GEPP_IR", "FP32_GMRES_IR",
                                    "BF16_GMRES_IR", "FP32_IR_SCALED"])
def test_solve_matches_oracle(ctx, name, mk, method):
    """Every method against the oracle; FP32_IR_SCALED factors the equilibrated
    matrix D_r A D_c."""
    scene = mk()
    pb, host = prepare(scene, 0.3)
    A_ref, b_ref = oracle_system(scene, host)
    ref = np.linalg.solve(A_ref, b_ref)
    scaled = method.endswith("_SCALED")
    method = method.replace("_SCALED", "")
    m = getattr(nrs, "NRS_" + method)
    sol, info = gpu_solve(ctx, scene, pb, host, m, equilibrate=int(scaled))
    ef, eg = rel_force_errors(sol, ref, scene["N"])
    assert ef <= 1e-8 and eg <= 1e-8, (ef, eg, info)
    assert info["fell_back"] == 0
    assert info["backward_error"] <= 1e-12
    if method != "FP64_LU":
        assert info["iterations"] >= 2
    if method.endswith("GMRES_IR"):
        assert info["method_used"] == getattr(nrs, "NRS_" + method)


def test_sphere_drag_on_gpu(ctx):
    scene = synth.sphere_scene(4, 16)
    pb, host = prepare(scene)
    sol, _ = gpu_solve(ctx, scene, pb, host, nrs.NRS_FP32_IR)
    W = oracle.patch_weights(host["w"], host["nu"], scene["N"])
    F = (W * sol[:scene["N"]]).sum()
    assert abs(F / (6 * math.pi) - 1) < 0.02


def test_c2_full_size_parity(ctx):
    """25 filaments (n = 3150), the time-stepping workload, full parity."""
    scene = synth.filament_scene(25, seed=0)
    pb, host = prepare(scene, 0.0)
    A_ref, b_ref = oracle_system(scene, host)
    ref = np.linalg.solve(A_ref, b_ref)
    for m in (nrs.NRS_FP64_LU, nrs.NRS_FP32_IR):
        sol, info = gpu_solve(ctx, scene, pb, host, m)
        ef, eg = rel_force_errors(sol, ref, scene["N"])
        assert ef <= 1e-8 and eg <= 1e-8, (m, ef, eg, info)


def test_solve_is_deterministic(ctx):
    scene = synth.filament_scene(5, seed=2)
    pb, host = prepare(scene, 1.1)
    s1, _ = gpu_solve(ctx, scene, pb, host, nrs.NRS_FP32_IR)
    s2, _ = gpu_solve(ctx, scene, pb, host, nrs.NRS_FP32_IR)
    np.testing.assert_array_equal(s1, s2)


@pytest.mark.parametrize("method", ["FP64_LU", "FP32_IR", "FP32_IR_REUSE"])
def test_rk4_step_matches_oracle(ctx, method):
    """Two RK4 steps against the oracle; FP32_IR_REUSE: stages 2-4 refine
    against the first stage's factors (reuse_stage_factors)."""
    scene = synth.filament_scene(5, seed=0)
    ds = nrs.DeviceScene(scene)
    reuse = method.endswith("_REUSE")
    m = getattr(nrs, "NRS_" + method.replace("_REUSE", ""))
    ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
    Y = T(scene["Y0"])
    Yo = scene["Y0"].copy()
    dt = 2 * math.pi / 100
    for step in range(2):
        nrs.nrs_rk4_step(ctx, ds, Y, step * dt, dt, ws, method=m, reuse_stage_factors=int(reuse))
        Yo = oracle.rk4_step(scene, Yo, step * dt, dt)
    info = nrs.nrs_query_info(ctx, ws)
    assert info["fell_back"] == 0
    err = np.max(np.abs(Y.cpu().numpy().reshape(-1, 12) - Yo))
    assert err <= 1e-10, err


@pytest.mark.parametrize("method", ["FP32_IR", "FP64_LU", "FP32_IR_REUSE"])
def test_rk4_headline_trajectory_matches_oracle(ctx, method):
    """The benchmark workload (25 filaments, n = 3150): two RK4 steps at
    dt = 2 pi / 100 against the oracle's states after each step, stored by
    tests/golden/make_golden.py (every oracle stage a full FP64 solve)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "rk4_filaments_M25_2steps.npz")
    with np.load(path, allow_pickle=False) as z:
        gold = [z["Y1"], z["Y2"]]
        dt = float(z["dt"])
    scene = synth.filament_scene(25, seed=0)
    ds = nrs.DeviceScene(scene)
    reuse = method.endswith("_REUSE")
    m = getattr(nrs, "NRS_" + method.replace("_REUSE", ""))
    ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
    Y = T(scene["Y0"])
    for step in range(2):
        nrs.nrs_rk4_step(ctx, ds, Y, step * dt, dt, ws, method=m, reuse_stage_factors=int(reuse))
        info = nrs.nrs_query_info(ctx, ws)
        assert info["fell_back"] == 0, (step, info)
        err = np.max(np.abs(Y.cpu().numpy().reshape(-1, 12) - gold[step]))
        print(f"rk4 M=25 {method} step {step + 1}: max state error {err:.2e}", flush=True)
        assert err <= 1e-10, (step, err)


def test_rk4_refinement_queue(ctx):
    """The refinement sweeps an RK4 step queues per stage (nrs_options.
    ir_queue): the adaptive default (the previous step's need plus one), a
    queue of one sweep under a tolerance that needs two (the step is redone
    with max_refine sweeps, no FP64 fallback) and the full queue of
    max_refine give bit-identical states (five filaments, n = 630, four
    steps each)."""
    scene = synth.filament_scene(5, seed=0)
    ds = nrs.DeviceScene(scene)
    m = nrs.NRS_FP32_IR
    dt = 2 * math.pi / 100

    def run(tol, queue):
        ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
        Y = T(scene["Y0"])
        its = []
        for step in range(4):
            nrs.nrs_rk4_step(ctx, ds, Y, step * dt, dt, ws, method=m, tol=tol, max_refine=4,
                             ir_queue=queue)
            info = nrs.nrs_query_info(ctx, ws)
            assert info["fell_back"] == 0, (tol, queue, step, info)
            its.append(info["iterations"])
        return Y.cpu().numpy(), its

    for tol in (0.0, 1e-13):
        full, its_full = run(tol, 4)
        adaptive, its_adapt = run(tol, 0)
        one, its_one = run(tol, 1)
        print(f"tol {tol}: updates per stage {its_full} / {its_adapt} / {its_one}", flush=True)
        assert its_adapt == its_full and its_one == its_full
        assert np.array_equal(adaptive, full) and np.array_equal(one, full)
    # the tight tolerance needs two corrections per stage, so the one-sweep
    # queue went through the redo
    assert max(its_full) >= 3, its_full
    with pytest.raises(nrs.NrsError, match="ir_queue"):
        ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
        nrs.nrs_rk4_step(ctx, ds, T(scene["Y0"]), 0.0, dt, ws, method=m, ir_queue=-1)


def test_rk4_stage_factor_reuse_at_headline_size(ctx):
    """25 filaments (n = 3150): three RK4 steps with stages 2-4 refined
    against the first stage's factors agree with refactoring every stage to
    the refinement tolerance, with no fallback; the option is ignored by the
    FP64 method."""
    scene = synth.filament_scene(25, seed=0)
    ds = nrs.DeviceScene(scene)
    m = nrs.NRS_FP32_IR
    ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
    dt = 2 * math.pi / 100
    Ys = []
    for reuse in (0, 1):
        Y = T(scene["Y0"])
        for step in range(3):
            nrs.nrs_rk4_step(ctx, ds, Y, step * dt, dt, ws, method=m, reuse_stage_factors=reuse)
            info = nrs.nrs_query_info(ctx, ws)
            assert info["fell_back"] == 0, (reuse, step, info)
        Ys.append(Y.cpu().numpy())
    err = np.abs(Ys[0] - Ys[1]).max()
    assert err <= 1e-10, err
    Y64 = [T(scene["Y0"]), T(scene["Y0"])]
    for reuse, Yd in zip((0, 1), Y64):
        nrs.nrs_rk4_step(ctx, ds, Yd, 0.0, dt, ws, method=nrs.NRS_FP64_LU,
                         reuse_stage_factors=reuse)
    np.testing.assert_array_equal(Y64[0].cpu().numpy(), Y64[1].cpu().numpy())


def test_errors_are_reported(ctx):
    scene = synth.filament_scene(1, seed=0)
    pb, host = prepare(scene)
    ws = workspace(ctx, pb, nrs.NRS_FP32_IR)
    sol = torch.empty(pb.n, dtype=torch.float64, device=DEV)
    with pytest.raises(nrs.NrsError, match="workspace"):
        nrs.nrs_solve(ctx, pb, T(host["u"]), None, sol, ws[:1000], method=nrs.NRS_FP32_IR)
    bad = nrs.Problem(pb.x, pb.X, pb.w, T(np.full(pb.Q, pb.N + 3), torch.int32), pb.body, pb.Y,
                      pb.eps, pb.mu)
    with pytest.raises(nrs.NrsError, match="invalid argument"):
        nrs.nrs_solve(ctx, bad, T(host["u"]), None, sol, ws, method=nrs.NRS_FP32_IR)
    xn = host["x"].copy()
    xn[0, 3] = np.nan
    pbn = nrs.Problem(T(xn), pb.X, pb.w, pb.nu, pb.body, pb.Y, pb.eps, pb.mu)
    with pytest.raises(nrs.NrsError, match="non-finite"):
        nrs.nrs_solve(ctx, pbn, T(host["u"]), None, sol, ws, method=nrs.NRS_FP64_LU)
    with pytest.raises(nrs.NrsError, match="invalid argument"):
        nrs.nrs_solve(ctx, nrs.Problem(pb.x, pb.X, pb.w, pb.nu, pb.body, pb.Y, -1.0, 1.0),
                      T(host["u"]), None, sol, ws)
    with pytest.raises(ValueError):
        nrs.nrs_solve(ctx, pb, torch.from_numpy(host["u"].ravel()), None, sol, ws)


def test_minimal_problem(ctx):
    """One force point, one quadrature point: A = (8 pi mu)^-1 S^eps(0) w."""
    x = np.array([[0.3], [0.1], [-0.2]])
    pb = nrs.Problem(T(x), T(x.copy()), T(np.array([0.5])), T(np.array([0]), torch.int32),
                     T(np.array([-1]), torch.int32), None, 0.1, 2.0)
    ws = workspace(ctx, pb, nrs.NRS_FP32_IR)
    sol = torch.empty(3, dtype=torch.float64, device=DEV)
    u = np.array([1.0, -2.0, 0.5])
    nrs.nrs_solve(ctx, pb, T(u), None, sol, ws, method=nrs.NRS_FP32_IR)
    a = 0.5 * (2.0 / 0.1) / (8 * math.pi * 2.0)
    np.testing.assert_allclose(sol.cpu().numpy(), u / a, rtol=1e-12)


@pytest.mark.parametrize("name,mk", [("filaments_M5", lambda: synth.filament_scene(5, seed=0)),
                                     ("rodwall_1500", lambda: synth.rod_wall_batch(1, seed=5, lo=1500, hi=1500)[0])])
def test_autotune_never_changes_results(ctx, name, mk):
    """The assembly launch shape chosen by the autotuner is recorded for the
    size class and used afterwards; matrices and solutions are bit-identical
    to those of the default shape."""
    scene = mk()
    pb, host = prepare(scene, 0.1)
    ws = workspace(ctx, pb, nrs.NRS_FP32_IR)
    lda = nrs.lda_for(pb.n)
    nrs.nrs_autotune_clear(ctx)

    def run():
        A32 = torch.zeros((pb.n, lda), dtype=torch.float32, device=DEV)
        A64 = torch.zeros((pb.n, lda), dtype=torch.float64, device=DEV)
        nrs.nrs_assemble(ctx, pb, 32, A32, lda, ws)
        nrs.nrs_assemble(ctx, pb, 64, A64, lda, ws)
        sol, info = gpu_solve(ctx, scene, pb, host, nrs.NRS_FP32_IR)
        return A32, A64, sol

    A32, A64, sol = run()
    res = nrs.nrs_autotune(ctx, pb, ws)
    assert res["block32"] in (64, 128, 256) and res["strip32"] in (4, 8, 16)
    assert res["block64"] in (64, 128, 256) and res["strip64"] in (4, 8, 16)
    assert 0 < res["ms32"] <= res["default_ms32"] and 0 < res["ms64"] <= res["default_ms64"]
    B32, B64, sol2 = run()
    assert torch.equal(A32, B32) and torch.equal(A64, B64)
    np.testing.assert_array_equal(sol, sol2)
    nrs.nrs_autotune_clear(ctx)
