"""rbcg_op_apply_noalloc: the block product with every device buffer carved
from the library's fixed per-GPU scratch array (no allocation), checked
against rbcg_op_apply on the same inputs and against the exact product of
the same rounded operands (bounds of the block-product unit test: FP64
1e-13, FP32 2e-5).  Two calls in a row, the second smaller, so the second
runs on whatever the first left in the shared array."""
import numpy as np
import pytest

import synth
from gpu_util import note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18717_amd import rbcg
    return rbcg, rbcg.Context()


def _rel(W, ref):
    return np.abs(W - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("matvec", ["f64", "f32"])
def test_noalloc_matches_op_apply_two_calls(R, matvec):
    import torch
    rbcg, ctx = R
    for d, N in ((8192, 65), (1000, 17)):
        note(f"noalloc {matvec} d={d} N={N}")
        P = synth.dense_problem(1, d, 1.5, 4, 1e-3)
        A = P["A"]
        X = synth.rng(21, 0).standard_normal((N, d))
        X[N // 3] = 0.0
        op = rbcg.DenseOperator(ctx, to_dev(A), lo="f32")
        Xd = to_dev(X)
        W1 = torch.full((N, d), float("nan"), dtype=torch.float64, device="cuda")
        W2 = torch.full((N, d), float("nan"), dtype=torch.float64, device="cuda")
        rbcg.op_apply(ctx, op, Xd, W1, matvec)
        ws_before = ctx.workspace_bytes()
        rbcg.op_apply_noalloc(ctx, op, Xd, W2, matvec)
        assert ctx.workspace_bytes() == ws_before
        w1, w2 = W1.cpu().numpy(), W2.cpu().numpy()
        if matvec == "f64":
            ref, bound = X @ A.T, 1e-13
        else:
            ref = X.astype(np.float32).astype(np.float64) @ A.astype(np.float32).astype(np.float64).T
            bound = 2e-5
        e1, e2 = _rel(w1, ref), _rel(w2, ref)
        note(f"  op_apply {e1:.2e}, noalloc {e2:.2e}, max |noalloc - op_apply| {np.abs(w2 - w1).max():.2e}")
        assert e2 <= bound
        assert _rel(w2, w1) <= bound
        del op


def test_noalloc_rejects_oversize(R):
    import torch
    rbcg, ctx = R
    cap = rbcg.noalloc_scratch_bytes()
    d, N = 16384, 256      # basis slots and partials far beyond the fixed array
    assert 2 * N * d * 8 > cap
    A = torch.eye(d, dtype=torch.float64, device="cuda")
    op = rbcg.DenseOperator(ctx, A)
    X = torch.zeros((N, d), dtype=torch.float64, device="cuda")
    W = torch.zeros((N, d), dtype=torch.float64, device="cuda")
    with pytest.raises(rbcg.RbcgError) as ei:
        rbcg.op_apply_noalloc(ctx, op, X, W, "f64")
    assert ei.value.code == -8
