"""nrs_lu_solve_noalloc (the triangular solves on the library's static scratch,
for callers that cannot allocate) against nrs_lu_solve on the same factors:
bit-identical solutions (same kernels, same arithmetic), for two calls in a
row with the second smaller than the first, in FP32 with static block
pivoting and in FP64 with partial pivoting; sizes past the scratch's limit
are refused."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2001_06468_amd as nrs
    from gpu_util import DEV, T, lu_ws, lus_ws


def _factor(ctx, A0, dt, scope):
    n = A0.shape[0]
    A = torch.from_numpy(A0.T.copy()).to(dt).to(DEV)
    ipiv = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    sing = torch.zeros(1, dtype=torch.int32, device=DEV)
    nrs.nrs_lu_factor(ctx, A, n, ipiv, perm, sing, lu_ws(ctx, n, A), pivot_scope=scope)
    assert sing.item() == 0
    return A, perm


@pytest.mark.parametrize("dt,scope", [(torch.float32, 1), (torch.float64, 0)],
                         ids=["fp32-block-pivots", "fp64-partial-pivots"])
def test_noalloc_solve_matches_workspace_solve(dt, scope):
    ctx = nrs.Context(0)
    rng = np.random.default_rng(7)
    for n in (3150, 515):                     # the second call is smaller
        A0 = rng.normal(size=(n, n)) + 3 * np.sqrt(n) * np.eye(n)
        b = rng.normal(size=n)
        A, perm = _factor(ctx, A0, dt, scope)
        bd = T(b, dt)
        x_ws = torch.empty(n, dtype=dt, device=DEV)
        x_na = torch.full((n,), float("nan"), dtype=dt, device=DEV)
        nrs.nrs_lu_solve(ctx, A, n, perm, bd, x_ws, lus_ws(ctx, n), pivot_scope=scope)
        nrs.nrs_lu_solve_noalloc(ctx, A, n, perm, bd, x_na, pivot_scope=scope)
        assert nrs.nrs_lu_query(ctx) == 0
        assert torch.equal(x_ws, x_na), n
        ref = np.linalg.solve(A0, b)
        tol = 1e-4 if dt == torch.float32 else 1e-10
        assert np.linalg.norm(x_na.cpu().numpy() - ref) / np.linalg.norm(ref) < tol, n
    ctx.close()


def test_noalloc_solve_limit():
    ctx = nrs.Context(0)
    n = nrs.NRS_NOALLOC_MAX_N + 1
    LU = torch.zeros(1, dtype=torch.float32, device=DEV)
    perm = torch.zeros(n, dtype=torch.int32, device=DEV)
    b = torch.zeros(1, dtype=torch.float32, device=DEV)
    x = torch.zeros(1, dtype=torch.float32, device=DEV)
    with pytest.raises(nrs.NrsError, match="NRS_NOALLOC_MAX_N"):
        nrs.nrs_lu_solve_noalloc(ctx, LU, n, perm, b, x, pivot_scope=1)
    ctx.close()
