"""Pins of the block-preconditioner oracle (oracle/precond.py): the
trigonometric fit against polynomials it must reproduce exactly, the rotation
covariance of a body's diagonal block (an invariant of the Sec. 3 eq. 23
operator and of the rigid-body rows of Sec. 4), and the preconditioner as an
exact inverse on block-diagonal matrices."""
import math

import numpy as np

import oracle
from oracle import precond as P
import synth


def test_trig_fit_reproduces_trigonometric_polynomials():
    rng = np.random.default_rng(3)
    H = 4
    coef = rng.normal(size=(2 * H + 1, 3, 2))
    for psis in (rng.uniform(0, 2 * math.pi, size=17),          # scattered phases
                 2 * math.pi * np.arange(2 * H + 1) / (2 * H + 1)):  # the fewest equispaced
        samples = np.stack([np.tensordot(P.trig_basis(p, H)[0], coef, axes=1) for p in psis])
        got = P.trig_fit(samples, psis, H)
        assert np.max(np.abs(got - coef)) < 1e-12
        psi = 0.7
        direct = coef[0] + sum(coef[2 * h - 1] * math.cos(h * psi) + coef[2 * h] * math.sin(h * psi)
                               for h in range(1, H + 1))
        assert np.max(np.abs(P.trig_eval(got, psi, H) - direct)) < 1e-12


def test_trig_fit_of_equispaced_samples_is_the_discrete_fourier_sum():
    # on S >= 2H + 1 equispaced phases the basis columns are orthogonal:
    # C_0 = mean, C_ch = (2/S) sum cos(h psi_s) K_s, C_sh = (2/S) sum sin(h psi_s) K_s
    rng = np.random.default_rng(4)
    S, H = 12, 3
    psis = 2 * math.pi * np.arange(S) / S
    K = rng.normal(size=(S, 5))
    got = P.trig_fit(K, psis, H)
    assert np.allclose(got[0], K.mean(axis=0), atol=1e-13)
    for h in range(1, H + 1):
        assert np.allclose(got[2 * h - 1], 2 / S * np.cos(h * psis) @ K, atol=1e-13)
        assert np.allclose(got[2 * h], 2 / S * np.sin(h * psis) @ K, atol=1e-13)


def test_body_block_is_the_rotated_block_of_the_body_alone():
    """Body b's diagonal block of a 3-filament scene equals R_b A_1(psi_b) R_b^T,
    A_1 the block of one filament alone in its own frame at the same phase."""
    sc = synth.filament_scene(3, seed=2, Nf=12, Qf=96)
    one = synth.filament_scene(1, seed=0, Nf=12, Qf=96)
    t = 0.37
    Y = sc["Y0"]
    A = P.system_matrix(sc, t, Y)
    blocks = P.diagonal_blocks(A, sc["N"], sc["M"], sc["body"])
    for b in range(sc["M"]):
        psi = P.body_phase(sc, b, t)
        A1 = P.one_body_blocks(one, [psi])[0]
        R = P.frame_rotation(np.asarray(Y[b, 3:]).reshape(3, 3), 12)
        ref = R @ A1 @ R.T
        assert np.max(np.abs(blocks[b] - ref)) <= 1e-12 * np.max(np.abs(ref))
    # a different phase gives a different block (the phase is what the model learns)
    A2 = P.one_body_blocks(one, [P.body_phase(sc, 0, t) + 0.5])[0]
    R0 = P.frame_rotation(np.asarray(Y[0, 3:]).reshape(3, 3), 12)
    assert np.max(np.abs(blocks[0] - R0 @ A2 @ R0.T)) > 1e-3 * np.max(np.abs(A2))


def test_frame_rotation_is_orthogonal_and_maps_vectors():
    rng = np.random.default_rng(5)
    B = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    R = P.frame_rotation(B, 4)
    assert np.allclose(R @ R.T, np.eye(18), atol=1e-14)
    v = rng.normal(size=18)
    z = R @ v
    assert np.allclose(z[[1, 5, 9]], B @ v[[1, 5, 9]], atol=1e-14)      # point 1
    assert np.allclose(z[15:18], B @ v[15:18], atol=1e-14)              # Omega


def test_preconditioner_inverts_a_block_diagonal_matrix():
    rng = np.random.default_rng(6)
    N, M = 7, 2
    body = np.array([0, 0, 0, 1, 1, -1, -1])
    n = 3 * N + 6 * M
    A = np.eye(n)
    blocks = []
    for b in range(M):
        r = P.body_rows(N, body, b)
        Bk = rng.normal(size=(len(r), len(r))) + 4 * np.eye(len(r))
        A[np.ix_(r, r)] = Bk
        blocks.append(Bk)
    got = P.diagonal_blocks(A, N, M, body)
    for g, Bk in zip(got, blocks):
        assert np.array_equal(g, Bk)
    v = rng.normal(size=n)
    z = P.apply_block_preconditioner(P.block_inverses(got), N, body, v)
    assert np.allclose(z, np.linalg.solve(A, v), rtol=1e-12, atol=1e-12)


def test_body_rows_order():
    body = np.array([1, 0, 0, 1])
    r = P.body_rows(4, body, 0)
    assert r.tolist() == [1, 2, 5, 6, 9, 10, 12, 13, 14, 15, 16, 17]
