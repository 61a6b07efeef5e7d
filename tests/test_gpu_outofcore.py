"""Host-resident (streamed) dense operator, the out-of-core setting of the
paper's wall-clock experiment (Sec. 7.1.1, intro figure: A is held in row
chunks, and every block product loads each chunk once).  Through the C ABI:

- rbcg_op_apply streams A in chunks of `chunk_rows` rows; the product must
  equal the exact FP64 product to 1e-13 (relative, max norm) for ragged chunk
  counts, an odd leading dimension (no 16-byte rows), widths across the
  column-chunk boundary of 144, and a single chunk; the streamed FP32 copy
  gives fl32(A) fl32(X) to 2e-5;
- mixed precision with streamed FP32 chunks and FP64 refinement reaches
  rtol 1e-10 and the dense solution to 1e-8;
- rbcg_solve with the streamed operator gives the oracle's bcg_t (eq. bcg_alg)
  to the plain-FP64 bound max(1e-12, 0.1 kappa u), converges to rtol exactly
  as the device-resident operator does, and also runs batched beside a
  device-resident system;
- Nystrom PCG (Sec. 2.2.2) with the streamed operator reproduces the
  preconditioned-CG definition to 1e-9, as with the device operator;
- the ridge-type path and the (inverse) square root with the streamed operator
  give the device-resident operator's results;
- FP32 products without the handle's FP32 copy are rejected
  (RBCG_ERR_UNSUPPORTED), and so is pageable host memory (RBCG_ERR_INVALID_ARG).
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import block_cg as ob
from oracle import krylov as ok
from oracle import truth as ot

from gpu_util import a_err, fp64_bound, note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18717_amd import rbcg
    return rbcg, rbcg.Context()


def _pinned(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A)).pin_memory()


@pytest.mark.parametrize("d,chunk,N", [(777, 100, 1), (777, 100, 17), (777, 100, 65), (777, 100, 130),
                                       (777, 250, 200), (1024, 1024, 33), (1000, 64, 129)])
def test_streamed_block_product(R, d, chunk, N):
    import torch
    rbcg, ctx = R
    note(f"streamed op_apply d={d} chunk={chunk} N={N}")
    A = synth.dense_problem(3, d, 1.0, 4, 1e-3)["A"]
    X = synth.rng(5, 0).standard_normal((N, d))
    X[N // 3: N // 3 + N // 4] = 0.0
    op = rbcg.DenseHostOperator(ctx, _pinned(A), chunk)
    W = torch.full((N, d), float("nan"), dtype=torch.float64, device="cuda")
    rbcg.op_apply(ctx, op, to_dev(X), W, "f64")
    ref = X @ A.T
    err = np.abs(W.cpu().numpy() - ref).max() / np.abs(ref).max()
    note(f"  rel err {err:.2e}")
    assert err <= 1e-13
    # the fixed-scratch entry point streams through the handle's own staging buffer
    W.fill_(float("nan"))
    if N <= 65:
        rbcg.op_apply_noalloc(ctx, op, to_dev(X), W, "f64")
        err2 = np.abs(W.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err2 <= 1e-13


@pytest.mark.parametrize("d,chunk,N", [(777, 100, 65), (777, 100, 17), (1000, 64, 129), (777, 250, 200)])
def test_streamed_fp32_block_product(R, d, chunk, N):
    """FP32 copy streamed from host memory: the product equals the exact product of the
    rounded operands fl32(A) fl32(X) to 2e-5 (FP32 accumulation), as the device-resident FP32
    product does."""
    import torch
    rbcg, ctx = R
    note(f"streamed f32 op_apply d={d} chunk={chunk} N={N}")
    A = synth.dense_problem(3, d, 1.0, 4, 1e-3)["A"]
    X = synth.rng(6, 0).standard_normal((N, d))
    op = rbcg.DenseHostOperator(ctx, _pinned(A), chunk, lo="f32")
    W = torch.full((N, d), float("nan"), dtype=torch.float64, device="cuda")
    rbcg.op_apply(ctx, op, to_dev(X), W, "f32")
    A32 = A.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    ref = X32 @ A32.T
    err = np.abs(W.cpu().numpy() - ref).max() / np.abs(ref).max()
    note(f"  rel err {err:.2e}")
    assert err <= 2e-5
    # the same handle still streams FP64 for FP64 products
    rbcg.op_apply(ctx, op, to_dev(X), W, "f64")
    ref64 = X @ A.T
    assert np.abs(W.cpu().numpy() - ref64).max() / np.abs(ref64).max() <= 1e-13


def test_streamed_mixed_solve_reaches_target(R):
    """FP32 chunks + FP64 refinement (FP64 residuals from the FP64 host matrix) reach rtol 1e-10
    and the dense solution to 1e-8 in the A_mu-norm, with the sweep and load counts of the
    device-resident mixed solve."""
    import torch
    rbcg, ctx = R
    P = synth.dense_problem(4, 1500, 1.5, 16, 1e-4)
    note("streamed mixed solve d=1500 chunk=256 k=16 rtol 1e-10")
    hop = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 256, lo="f32")
    dop = rbcg.DenseOperator(ctx, to_dev(P["A"]), lo="f32")
    b, om = to_dev(P["b"]), to_dev(P["omega"])
    o = rbcg.opts(60, rtol=1e-10, matvec="f32", refine_max=8)
    xh, xd = torch.zeros_like(b), torch.zeros_like(b)
    rc, ih = rbcg.solve(ctx, [hop], [P["mu"]], [b], [om], [xh], [o], check=False)
    assert rc == 0, ih
    rc, idv = rbcg.solve(ctx, [dop], [P["mu"]], [b], [om], [xd], [o], check=False)
    assert rc == 0, idv
    xt = ot.solve_dense(P["A"], P["mu"], P["b"])
    eh = a_err(P["A"], P["mu"], xh.cpu().numpy(), xt)
    note(f"  sweeps {ih[0]['refine_sweeps']} loads {ih[0]['matrix_loads']} relres {ih[0]['relres']:.2e} "
         f"err {eh:.2e}; device-resident sweeps {idv[0]['refine_sweeps']} loads {idv[0]['matrix_loads']}")
    assert ih[0]["relres"] <= 1e-10 and ih[0]["precision_used"] == 1
    assert eh <= 1e-8
    assert abs(ih[0]["matrix_loads"] - idv[0]["matrix_loads"]) <= 2


@pytest.fixture(scope="module")
def c_mid():
    return synth.dense_problem(4, 1500, 1.5, 16, 1e-4)


@pytest.mark.parametrize("t", [1, 6, 12])
def test_streamed_solve_iterates_match_oracle(R, c_mid, t):
    import torch
    rbcg, ctx = R
    P = c_mid
    note(f"streamed solve d=1500 chunk=256 k=16 t={t}")
    op = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 256)
    b = to_dev(P["b"])
    x = torch.zeros_like(b)
    rc, info = rbcg.solve(ctx, [op], [P["mu"]], [b], [to_dev(P["omega"])], [x], [rbcg.opts(t)], check=False)
    assert rc == 0, info
    assert info[0]["iters"] == t and info[0]["matrix_loads"] == t + 1   # + the FP64 residual product
    X, _ = ob.bcg(P["A"], [P["mu"]], P["b"], P["omega"], t)
    lam = np.linalg.eigvalsh(P["A"])
    kappa = (lam[-1] + P["mu"]) / (lam[0] + P["mu"])
    err = a_err(P["A"], P["mu"], x.cpu().numpy(), X[0])
    note(f"  vs oracle {err:.2e} (bound {fp64_bound(kappa):.1e})")
    assert err <= fp64_bound(kappa)


def test_streamed_solve_to_rtol_and_batched_beside_device_operator(R, c_mid):
    import torch
    rbcg, ctx = R
    P = c_mid
    Q = synth.dense_problem(5, 900, 2.0, 8, 1e-3)
    note("streamed solve d=1500 rtol 1e-10, batched with a device-resident d=900 system")
    hop = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 500)
    dop = rbcg.DenseOperator(ctx, to_dev(P["A"]))
    qop = rbcg.DenseOperator(ctx, to_dev(Q["A"]))
    b, om = to_dev(P["b"]), to_dev(P["omega"])
    o = rbcg.opts(60, rtol=1e-10)
    xh, xd = torch.zeros_like(b), torch.zeros_like(b)
    rc, ih = rbcg.solve(ctx, [hop], [P["mu"]], [b], [om], [xh], [o], check=False)
    assert rc == 0, ih
    rc, idv = rbcg.solve(ctx, [dop], [P["mu"]], [b], [om], [xd], [o], check=False)
    assert rc == 0, idv
    assert ih[0]["relres"] <= 1e-10 and ih[0]["iters"] == idv[0]["iters"]
    diff = a_err(P["A"], P["mu"], xh.cpu().numpy(), xd.cpu().numpy())
    note(f"  iters {ih[0]['iters']}, streamed vs device-resident {diff:.2e}")
    assert diff <= 1e-11
    # two systems in one call: the streamed one and a device-resident one
    qb = to_dev(Q["b"])
    xh.zero_()
    xq = torch.zeros_like(qb)
    rc, ib = rbcg.solve(ctx, [hop, qop], [P["mu"], Q["mu"]], [b, qb], [om, to_dev(Q["omega"])], [xh, xq],
                        [o, o], check=False)
    assert rc == 0, ib
    assert ib[0]["relres"] <= 1e-10 and ib[1]["relres"] <= 1e-10
    assert a_err(P["A"], P["mu"], xh.cpu().numpy(), xd.cpu().numpy()) <= 1e-9


def test_two_systems_share_one_streamed_operator(R, c_mid):
    """Two right-hand sides of one streamed operator in one call (their products take turns in
    the handle's staging buffers): both reach rtol and match the single-system solves."""
    import torch
    rbcg, ctx = R
    P = c_mid
    note("two systems on one streamed operator d=1500 chunk=300")
    op = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 300)
    b1 = to_dev(P["b"])
    b2 = to_dev(synth.rng(9, 1).standard_normal(1500))
    om = to_dev(P["omega"])
    o = rbcg.opts(60, rtol=1e-10)
    x1, x2 = torch.zeros_like(b1), torch.zeros_like(b1)
    rc, info = rbcg.solve(ctx, [op, op], [P["mu"], 10 * P["mu"]], [b1, b2], [om, om], [x1, x2], [o, o],
                          check=False)
    assert rc == 0, info
    assert info[0]["relres"] <= 1e-10 and info[1]["relres"] <= 1e-10
    for bb, mu, xb in ((b1, P["mu"], x1), (b2, 10 * P["mu"], x2)):
        xs = torch.zeros_like(bb)
        rc, _ = rbcg.solve(ctx, [op], [mu], [bb], [om], [xs], [o], check=False)
        assert rc == 0
        assert a_err(P["A"], mu, xb.cpu().numpy(), xs.cpu().numpy()) <= 1e-9


def test_streamed_nystrom_pcg_matches_definition(R):
    import torch
    rbcg, ctx = R
    P = synth.dense_problem(1, 512, 2.0, 10, 1e-3)
    A, mu, b = P["A"], P["mu"], P["b"]
    Om = P["omega"][:10]
    op = rbcg.DenseHostOperator(ctx, _pinned(A), 100)
    U, D = ok.nystrom(A, Om, 2)
    Pinv = ok.deflation_pinv(U, D, D.min(), mu)
    for t in (1, 4, 8):
        note(f"streamed nystrom pcg d=512 chunk=100 s=2 t={t}")
        x = torch.zeros(512, dtype=torch.float64, device="cuda")
        rc, info, _, _, _ = rbcg.nystrom_pcg(ctx, op, to_dev(b), to_dev(Om), 2, mu, x, rbcg.opts(t), check=False)
        assert rc == 0, info
        assert info["iters"] == t and info["matrix_loads"] == 2 + t + 1
        err = a_err(A, mu, x.cpu().numpy(), ok.pcg_definition(A, mu, b, Pinv, t))
        note(f"  vs pcg_def {err:.2e}")
        assert err < 1e-9


def test_streamed_path_and_sampling_match_device_operator(R):
    """The path (every shift) and the square root / inverse square root with the streamed
    operator give the device-resident operator's results: the same arithmetic, with products
    summed chunk by chunk (FP64 path at fixed t: 5e-12, about kappa u for kappa ~ 8e3; FP32
    chunks + FP64 refinement, both at rtol 1e-10: 1e-8; sampling: 1e-10 relative)."""
    import torch
    rbcg, ctx = R
    P = synth.dense_problem(6, 1200, 1.5, 16, 1e-4)
    mus = [1e-4, 1e-3, 1e-2, 1e-1]
    hop = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 256, lo="f32")
    dop = rbcg.DenseOperator(ctx, to_dev(P["A"]), lo="f32")
    b, om = to_dev(P["b"]), to_dev(P["omega"])
    for o, tol in ((rbcg.opts(12), 5e-12), (rbcg.opts(40, rtol=1e-10, matvec="f32", refine_max=8), 1e-8)):
        note(f"streamed path d=1200 chunk=256 L=4 matvec={o.matvec}")
        Xh = torch.zeros((len(mus), 1200), dtype=torch.float64, device="cuda")
        Xd = torch.zeros_like(Xh)
        rc, ih = rbcg.path(ctx, hop, b, om, mus, Xh, o, check=False)
        assert rc == 0, ih
        rc, idv = rbcg.path(ctx, dop, b, om, mus, Xd, o, check=False)
        assert rc == 0, idv
        worst = max(a_err(P["A"], mu, Xh[l].cpu().numpy(), Xd[l].cpu().numpy()) for l, mu in enumerate(mus))
        note(f"  streamed vs device-resident, worst shift {worst:.2e}")
        assert worst <= tol
    Bs = synth.rng(7, 2).standard_normal((40, 1200))
    for inverse in (False, True):
        fn = rbcg.invsqrt_apply if inverse else rbcg.sqrt_apply
        note(f"streamed {'inverse ' if inverse else ''}square root, 40 samples in groups of 16")
        Yh = torch.zeros((40, 1200), dtype=torch.float64, device="cuda")
        Yd = torch.zeros_like(Yh)
        rc, _ = fn(ctx, hop, to_dev(Bs), Yh, rbcg.opts(10, nquad=16, group=16), check=False)
        assert rc == 0
        rc, _ = fn(ctx, dop, to_dev(Bs), Yd, rbcg.opts(10, nquad=16, group=16), check=False)
        assert rc == 0
        rel = float((torch.linalg.norm(Yh - Yd, dim=1) / torch.linalg.norm(Yd, dim=1)).max())
        note(f"  streamed vs device-resident {rel:.2e}")
        assert rel <= 1e-10


def test_streamed_operator_rejections(R):
    import torch
    rbcg, ctx = R
    P = synth.dense_problem(1, 256, 2.0, 4, 1e-3)
    op = rbcg.DenseHostOperator(ctx, _pinned(P["A"]), 64)
    b = to_dev(P["b"])
    om = to_dev(P["omega"])
    x = torch.zeros_like(b)
    rc, _ = rbcg.solve(ctx, [op], [1e-3], [b], [om], [x], [rbcg.opts(8, rtol=1e-8, matvec="f32", refine_max=3)],
                       check=False)
    assert rc == -7
    # pageable host memory: rejected before any copy
    Ah = np.ascontiguousarray(P["A"])
    h = ctypes.c_void_p()
    assert rbcg._op_dense_host(ctx.handle, ctypes.byref(h), 256, Ah.ctypes.data, 256, 64, 0) == -1
    # chunk sizes out of range
    Ap = _pinned(P["A"])
    assert rbcg._op_dense_host(ctx.handle, ctypes.byref(h), 256, Ap.data_ptr(), 256, 0, 0) == -1
    assert rbcg._op_dense_host(ctx.handle, ctypes.byref(h), 256, Ap.data_ptr(), 256, 257, 0) == -1
