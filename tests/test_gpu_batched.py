"""Batched uneven systems (nrs_solve_batched): every instance of a batch must
match its own single solve and the FP64 oracle.  Tolerances:
  batched vs single nrs_solve (same method) : bit-identical (the batch runs
    the same per-tile arithmetic, only the schedule differs);
  batched vs oracle : relative 2-norm error of forces and of (U, Omega)
    <= 1e-8.
The full-size case is the 512-instance rod-over-wall batch (orders drawn
log-uniformly in 300..6000), solved in the launch configuration the
benchmark times, 16 instances at evenly spaced ranks of the order checked
against FP64 oracle solutions stored by tests/golden/make_golden.py.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2001_06468_amd as nrs
    from gpu_util import T, prepare, oracle_system, workspace, rel_force_errors, DEV


@pytest.fixture(scope="module")
def ctx():
    c = nrs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _single(ctx, scene, pb, host):
    """The single solve of the same method (unscaled, as a batch)."""
    ws = workspace(ctx, pb, nrs.NRS_FP32_IR)
    sol = torch.empty(pb.n, dtype=torch.float64, device=DEV)
    ft = T(scene["ftext"]) if scene["M"] else None
    info = nrs.nrs_solve(ctx, pb, T(host["u"]), ft, sol, ws, method=nrs.NRS_FP32_IR)
    return sol.cpu().numpy(), info


def _batch(ctx, scenes, preps, info=True, ws=None):
    pbs = [p for p, _ in preps]
    us = [T(h["u"]) for _, h in preps]
    fts = [T(s["ftext"]) if s["M"] else None for s in scenes]
    sols = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in pbs]
    if ws is None:
        ws = torch.empty(nrs.nrs_solve_batched_workspace_size(ctx, pbs), dtype=torch.uint8,
                         device=DEV)
    infos = nrs.nrs_solve_batched(ctx, pbs, us, sols, ws, ftexts=fts, info=info)
    return [s.cpu().numpy() for s in sols], infos


def _mixed_scenes():
    """Uneven orders across tile boundaries, resistance and swimming problems."""
    rods = synth.rod_wall_batch(4, seed=7, lo=300, hi=1400)
    return [
        synth.filament_scene(1, seed=3),                 # n = 126, swimming
        rods[0],
        synth.sphere_scene(3, 9),                        # n = 162
        rods[1],
        synth.filament_scene(5, seed=1),                 # n = 630, swimming
        rods[2],
        synth.sphere_scene(3, 9, free=True, force=np.array([0, 0, -1.0])),
        rods[3],
    ]


def test_batched_matches_single_and_oracle(ctx):
    scenes = _mixed_scenes()
    preps = [prepare(s, 0.2) for s in scenes]
    sols, infos = _batch(ctx, scenes, preps)
    assert len({p.n for p, _ in preps}) == len(scenes)
    for k, (scene, (pb, host)) in enumerate(zip(scenes, preps)):
        single, sinfo = _single(ctx, scene, pb, host)
        assert infos[k]["fell_back"] == 0, (k, infos[k])
        np.testing.assert_array_equal(sols[k], single, err_msg=f"instance {k}, n = {pb.n}")
        A, b = oracle_system(scene, host)
        ref = np.linalg.solve(A, b)
        ef, eg = rel_force_errors(sols[k], ref, scene["N"])
        assert ef <= 1e-8 and eg <= 1e-8, (k, pb.n, ef, eg, infos[k])
        assert infos[k]["iterations"] == sinfo["iterations"]
        assert infos[k]["backward_error"] <= 1e-12


def _scatter_problem(N, seed, eps=0.05):
    """Resistance problem on N seeded points scattered over a unit sphere,
    8 quadrature points jittered around each force point (orders 3N chosen
    freely)."""
    rng = np.random.default_rng(seed)
    Q = 8 * N
    x = rng.normal(size=(3, N))
    x /= np.linalg.norm(x, axis=0)
    X = np.repeat(x, 8, axis=1) + 0.02 * rng.normal(size=(3, Q))
    X /= np.linalg.norm(X, axis=0)
    w = np.full(Q, 4 * np.pi / Q)
    nu = oracle.nearest(x, X, np.array([0, N]), np.zeros(Q, dtype=np.int32))
    assert np.bincount(nu, minlength=N).min() > 0   # every column of A_s nonzero
    u = rng.normal(size=(3, N))
    body = -np.ones(N, dtype=np.int32)
    pb = nrs.Problem(T(x), T(X), T(w), T(nu, torch.int32), T(body, torch.int32), None, eps, 1.0)
    As = oracle.assemble_As(x, X, w, nu, eps, 1.0)
    return pb, u, np.linalg.solve(As, u.ravel())


def test_batched_ragged_edges(ctx):
    """Orders 3 (one force point), 63, 66, 129 and 126 (swimming), and a
    one-instance batch."""
    x1 = np.array([[0.3], [0.1], [-0.2]])
    tiny = nrs.Problem(T(x1), T(x1.copy()), T(np.array([0.5])), T(np.array([0]), torch.int32),
                       T(np.array([-1]), torch.int32), None, 0.1, 2.0)
    u1 = np.array([1.0, -2.0, 0.5])
    a = 0.5 * (2.0 / 0.1) / (8 * np.pi * 2.0)
    probs, us, refs, fts = [tiny], [T(u1)], [u1 / a], [None]
    for N in (21, 22, 43):
        pb, u, ref = _scatter_problem(N, seed=N)
        probs.append(pb)
        us.append(T(u))
        refs.append(ref)
        fts.append(None)
    fil = synth.filament_scene(1, seed=5)
    pb, h = prepare(fil)
    A, b = oracle_system(fil, h)
    probs.append(pb)
    us.append(T(h["u"]))
    refs.append(np.linalg.solve(A, b))
    fts.append(T(fil["ftext"]))
    assert [p.n for p in probs] == [3, 63, 66, 129, 126]
    for subset in ([0], [3], list(range(len(probs)))):
        pbs = [probs[i] for i in subset]
        ws = torch.empty(nrs.nrs_solve_batched_workspace_size(ctx, pbs), dtype=torch.uint8,
                         device=DEV)
        sols = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in pbs]
        infos = nrs.nrs_solve_batched(ctx, pbs, [us[i] for i in subset], sols, ws,
                                      ftexts=[fts[i] for i in subset])
        for j, i in enumerate(subset):
            got = sols[j].cpu().numpy()
            N = probs[i].N
            ef, eg = rel_force_errors(got, refs[i], N)
            assert ef <= 1e-8 and eg <= 1e-8, (i, probs[i].n, ef, eg, infos[j])
            assert infos[j]["fell_back"] == 0


def test_batched_repeat_and_async(ctx):
    """Two calls in a row (synchronisation words self-clean) and the
    asynchronous form give identical results."""
    scenes = synth.rod_wall_batch(5, seed=11, lo=300, hi=900)
    preps = [prepare(s) for s in scenes]
    pbs = [p for p, _ in preps]
    ws = torch.empty(nrs.nrs_solve_batched_workspace_size(ctx, pbs), dtype=torch.uint8, device=DEV)
    s1, _ = _batch(ctx, scenes, preps, ws=ws)
    s2, _ = _batch(ctx, scenes, preps, ws=ws)
    s3, none = _batch(ctx, scenes, preps, ws=ws, info=False)
    assert none is None
    for a, b, c in zip(s1, s2, s3):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)


def test_batched_errors(ctx):
    scenes = synth.rod_wall_batch(2, seed=1, lo=300, hi=400)
    preps = [prepare(s) for s in scenes]
    pbs = [p for p, _ in preps]
    need = nrs.nrs_solve_batched_workspace_size(ctx, pbs)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    us = [T(h["u"]) for _, h in preps]
    sols = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in pbs]
    with pytest.raises(nrs.NrsError, match="unsupported"):
        nrs.nrs_solve_batched(ctx, pbs, us, sols, ws, method=nrs.NRS_FP64_LU)
    with pytest.raises(nrs.NrsError, match="workspace"):
        nrs.nrs_solve_batched(ctx, pbs, us, sols, ws[:need // 2])
    with pytest.raises(nrs.NrsError, match="invalid argument"):
        nrs.nrs_solve_batched(ctx, [], [], [], ws)
    bad = nrs.Problem(pbs[1].x, pbs[1].X, pbs[1].w,
                      T(np.full(pbs[1].Q, pbs[1].N + 2), torch.int32), pbs[1].body, None,
                      pbs[1].eps, pbs[1].mu)
    with pytest.raises(nrs.NrsError, match="problem 1"):
        nrs.nrs_solve_batched(ctx, [pbs[0], bad], us, sols, ws)


def device_batch(ctx, scenes, t=0.0):
    """Device problems of a list of resistance scenes, built by the library's
    own geometry and nearest-map entry points (the benchmark's inputs)."""
    probs, us = [], []
    for sc in scenes:
        ds = nrs.DeviceScene(sc, DEV)
        N, Q = sc["N"], sc["Q"]
        x = torch.empty(3 * N, dtype=torch.float64, device=DEV)
        X = torch.empty(3 * Q, dtype=torch.float64, device=DEV)
        w = torch.empty(Q, dtype=torch.float64, device=DEV)
        u = torch.empty(3 * N, dtype=torch.float64, device=DEV)
        nrs.nrs_geometry(ctx, ds, t, None, x, X, w, u)
        nu = torch.empty(Q, dtype=torch.int32, device=DEV)
        nrs.nrs_nearest(ctx, x.view(3, N), sc["group_off"], X.view(3, Q), ds.t["groupX"], nu)
        probs.append(nrs.Problem(x.view(3, N), X.view(3, Q), w, nu, ds.t["body"], None,
                                 sc["eps"], sc["mu"]))
        us.append(u)
    return probs, us


def test_c4_full_batch_sampled_parity(ctx):
    """All 512 rod-over-wall instances in one batched call; 16 instances
    spread over the size range against the oracle, every instance's FP64 backward error; six more calls
    on the same workspace give bit-identical solutions (a regression test of
    the tile LU's publish order: a tile's flag used to be able to overtake
    another wave's stores of that tile, which changed about one system's
    factors in 4,000 per call)."""
    scenes = synth.rod_wall_batch(512, seed=0)
    probs, us = device_batch(ctx, scenes)
    ns = np.array([p.n for p in probs])
    assert 300 * 0.9 <= ns.min() and ns.max() <= 6000 * 1.1
    ws = torch.empty(nrs.nrs_solve_batched_workspace_size(ctx, probs), dtype=torch.uint8,
                     device=DEV)
    sols = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in probs]
    infos = nrs.nrs_solve_batched(ctx, probs, us, sols, ws)
    bwd = np.array([i["backward_error"] for i in infos])
    assert all(i["fell_back"] == 0 for i in infos)
    assert bwd.max() <= 1e-12, bwd.max()
    first = torch.cat(sols).clone()
    for rep in range(6):
        nrs.nrs_solve_batched(ctx, probs, us, sols, ws, info=False)
        again = torch.cat(sols)
        bad = int((again != first).sum())
        assert bad == 0, (rep, bad)
    # 16 instances at evenly spaced ranks of n (303 ... 5868) against the
    # oracle's FP64 solutions stored by tests/golden/make_golden.py; the
    # nearest maps the library built must equal the oracle's, bit for bit
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "rodwall_B512_sample16.npz")
    with np.load(path, allow_pickle=False) as z:
        idx, gn, gsol, gdig = z["idx"], z["n"], z["sol"], z["nu_sha256"]
    assert len(idx) == 16 and gn.min() == ns.min() and gn.max() == ns.max()
    off = 0
    for k, nk, dig in zip(idx, gn, gdig):
        assert ns[k] == nk
        ref = gsol[off:off + nk]
        off += nk
        nu = probs[k].nu.cpu().numpy().astype(np.int32)
        assert hashlib.sha256(nu.tobytes()).hexdigest() == str(dig), k
        ef, _ = rel_force_errors(sols[k].cpu().numpy(), ref, scenes[k]["N"])
        assert ef <= 1e-8, (k, nk, ef, infos[k])


def test_batched_graph_replay():
    """The asynchronous batched solve captured into a HIP graph: every replay
    (with other GPU work and synchronisations in between) equals the eager
    solve bit for bit, and replays read the current contents of the inputs."""
    stream = torch.cuda.Stream()
    c = nrs.Context(0, stream=stream.cuda_stream)
    scenes = synth.rod_wall_batch(6, seed=21, lo=300, hi=1500)
    preps = [prepare(s) for s in scenes]
    pbs = [p for p, _ in preps]
    us = [T(h["u"]) for _, h in preps]
    ws = torch.empty(nrs.nrs_solve_batched_workspace_size(c, pbs), dtype=torch.uint8, device=DEV)
    sols_e = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in pbs]
    sols_g = [torch.empty(p.n, dtype=torch.float64, device=DEV) for p in pbs]
    torch.cuda.synchronize()
    nrs.nrs_solve_batched(c, pbs, us, sols_e, ws, info=False)
    stream.synchronize()
    ref = [x.clone() for x in sols_e]
    other = torch.randn(512, 512, device=DEV)
    for rep in range(3):
        for x in sols_g:
            x.zero_()
        (other @ other).sum().item()          # unrelated eager work between replays
        torch.cuda.synchronize()
        nrs.nrs_solve_batched(c, pbs, us, sols_g, ws, info=False, graph=1)
        stream.synchronize()
        for k in range(len(pbs)):
            assert torch.equal(sols_g[k], ref[k]), (rep, k)
    # new right-hand sides (same pointers): the replay solves for them; scaling
    # by two is exact through every step, so the result is exactly 2 x
    for u in us:
        u.mul_(2.0)
    torch.cuda.synchronize()
    nrs.nrs_solve_batched(c, pbs, us, sols_g, ws, info=False, graph=1)
    stream.synchronize()
    for k in range(len(pbs)):
        assert torch.equal(sols_g[k], 2.0 * ref[k]), k
    with pytest.raises(nrs.NrsError, match="asynchronous"):
        nrs.nrs_solve_batched(c, pbs, us, sols_g, ws, info=True, graph=1)
    c.close()
    # the default (null) stream cannot be captured
    c0 = nrs.Context(0, stream=0)
    with pytest.raises(nrs.NrsError, match="non-default stream"):
        nrs.nrs_solve_batched(c0, pbs, us, sols_g, ws, info=False, graph=1)
    c0.close()
