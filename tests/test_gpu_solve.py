"""GPU parity of rbcg_solve (through the C ABI) against the FP64 CPU oracle.

Tolerances: plain FP64 block-CG iterates must match the oracle's iterate at
the same t to a relative A_mu-norm difference of max(1e-12, 0.1 kappa u),
kappa = cond(A + mu I), u = 2^-53: two correct FP64 implementations that
round differently agree only to about kappa u on ill-conditioned systems
(measured against an extended-precision reference in test_gpu_batch.py).  Mixed precision with FP64 refinement must match
the converged oracle solution to 1e-8.
"""
import numpy as np
import pytest

import synth
from oracle import block_cg as ob
from oracle import truth as ot

from gpu_util import a_err, fp64_bound, note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18717_amd import rbcg
    ctx = rbcg.Context()
    return rbcg, ctx


def _solve_one(R, A, mu, b, Om, t, rtol=0.0, matvec="f64", refine=1, lo="f64"):
    import torch
    rbcg, ctx = R
    Ad = to_dev(A)
    op = rbcg.DenseOperator(ctx, Ad, lo=lo)
    bd = to_dev(b)
    om = to_dev(Om) if Om is not None and len(Om) else None
    x = torch.zeros_like(bd)
    o = rbcg.opts(t, rtol=rtol, matvec=matvec, refine_max=refine)
    rc, info = rbcg.solve(ctx, [op], [mu], [bd], [om], [x], [o], check=False)
    torch.cuda.synchronize()
    return rc, info[0], x.cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    return synth.dense_problem(1, 512, 2.0, 16, 1e-3)


@pytest.mark.parametrize("t", [1, 2, 5, 10, 30])
def test_c1_iterates_match_oracle(R, c1, t):
    """C1 (d=512, k=16, mu=1e-3): the GPU iterate after t block products is
    the oracle's bcg_t (eq. bcg_alg) to 1e-12 in the A_mu-norm."""
    note(f"c1 t={t}")
    rc, info, x = _solve_one(R, c1["A"], c1["mu"], c1["b"], c1["omega"], t)
    assert rc == 0, info
    X, _ = ob.bcg(c1["A"], [c1["mu"]], c1["b"], c1["omega"], t)
    assert info["iters"] == t
    err = a_err(c1["A"], c1["mu"], x, X[0])
    assert err < 1e-12, err


def test_c1_exact_termination(R, c1):
    """t = 31: 17 * 31 >= 512, the last block deflates; GPU equals the dense
    Cholesky solution."""
    note("c1 t=31 exact termination")
    rc, info, x = _solve_one(R, c1["A"], c1["mu"], c1["b"], c1["omega"], 31)
    assert rc == 0, info
    xt = ot.solve_dense(c1["A"], c1["mu"], c1["b"])
    assert a_err(c1["A"], c1["mu"], x, xt) < 1e-12


@pytest.mark.parametrize("d,k,t,p,mu", [(300, 7, 6, 1.0, 1e-2), (1000, 20, 4, 1.5, 1e-4), (129, 0, 12, 1.0, 1e-1),
                                         (777, 33, 3, 2.0, 0.0), (64, 63, 1, 1.0, 1e-3)])
def test_ragged_shapes(R, d, k, t, p, mu):
    """Ragged d (not tile multiples), k = 0 (plain CG), mu = 0 and a full first block."""
    note(f"ragged d={d} k={k} t={t}")
    g = np.random.default_rng(d + k)
    lam = np.arange(1, d + 1, dtype=float) ** (-p)
    A = synth.spd_from_spectrum(lam, g)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    rc, info, x = _solve_one(R, A, mu, b, Om, t)
    assert rc == 0, info
    X, _ = ob.bcg(A, [mu], b, Om if k else None, t)
    kappa = (lam[0] + mu) / (lam[-1] + mu)
    assert a_err(A, mu, x, X[0]) < fp64_bound(kappa)


@pytest.mark.parametrize("d,k,t", [(200, 128, 2), (150, 64, 3)])
def test_deflation_late_in_a_block(R, d, k, t):
    """The Krylov space reaches dimension d partway through the last block (129 + 71 = 200,
    2 * 65 + 20 = 150): that block's factorization starts unpivoted, completes several rows of
    its output, then meets a deflated column and is redone with pivoting by the same
    workgroup.  Exact termination: the answer is the dense solution."""
    note(f"late deflation d={d} k={k} t={t}")
    g = np.random.default_rng(7 * d + k)
    lam = np.arange(1, d + 1, dtype=float) ** (-1.0)
    A = synth.spd_from_spectrum(lam, g)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    mu = 1e-2
    rc, info, x = _solve_one(R, A, mu, b, Om, t)
    assert rc == 0, info
    assert info["deflated"] > 0, info
    xt = ot.solve_dense(A, mu, b)
    assert a_err(A, mu, x, xt) < 1e-11


def test_batched_uneven_systems_match_one_at_a_time(R):
    """Several systems of uneven d and k in one call equal separate calls and
    the oracle (batching must not change results)."""
    import torch
    rbcg, ctx = R
    note("batched 3 systems")
    probs = []
    for i, (d, k, p, mu) in enumerate([(400, 8, 1.2, 1e-3), (1100, 16, 2.0, 1e-5), (257, 31, 1.0, 1e-2)]):
        g = np.random.default_rng(100 + i)
        lam = np.arange(1, d + 1, dtype=float) ** (-p)
        A = synth.spd_from_spectrum(lam, g)
        probs.append((A, mu, g.standard_normal(d), g.standard_normal((k, d)), (1.0 + mu) / (lam[-1] + mu)))
    t = 6
    ops = [rbcg.DenseOperator(ctx, to_dev(A)) for A, *_ in probs]
    bs = [to_dev(pr[2]) for pr in probs]
    oms = [to_dev(pr[3]) for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    o = [rbcg.opts(t) for _ in probs]
    rc, info = rbcg.solve(ctx, ops, [pr[1] for pr in probs], bs, oms, xs, o)
    assert rc == 0
    for (A, mu, b, Om, kappa), xd in zip(probs, xs):
        X, _ = ob.bcg(A, [mu], b, Om, t)
        assert a_err(A, mu, xd.cpu().numpy(), X[0]) < 1e-11
        # alone, the system gets a different split-K partition and, when its block width is
        # one the exact-width factorization kernel serves, a different kernel (pivot ties may
        # break differently): equal up to rounding, at the oracle-parity bound
        rc1, _, x1 = _solve_one(R, A, mu, b, Om, t)
        assert a_err(A, mu, x1, xd.cpu().numpy()) < fp64_bound(kappa)


def test_rtol_stops_and_reports_relres(R):
    note("rtol fp64")
    g = np.random.default_rng(5)
    d = 1500
    A = synth.spd_from_spectrum(np.arange(1, d + 1, dtype=float) ** (-1.5), g)
    b = g.standard_normal(d)
    Om = g.standard_normal((24, d))
    rc, info, x = _solve_one(R, A, 1e-4, b, Om, 60, rtol=1e-10, refine=2)
    assert rc == 0, info
    r = b - (A @ x + 1e-4 * x)
    relres = np.linalg.norm(r) / np.linalg.norm(b)
    assert relres <= 1e-10
    assert abs(relres - info["relres"]) <= 1e-3 * relres + 1e-16
    assert info["iters"] < 60


def test_mixed_f32_refinement_matches_oracle(R):
    """FP32 MFMA block products with FP64 refinement reach the FP64 answer:
    relative A_mu-norm error <= 1e-8 against the dense oracle solution."""
    note("mixed f32 refine d=2048")
    g = np.random.default_rng(6)
    d = 2048
    A = synth.spd_from_spectrum(np.arange(1, d + 1, dtype=float) ** (-1.5), g)
    b = g.standard_normal(d)
    Om = g.standard_normal((64, d))
    mu = 1e-4
    rc, info, x = _solve_one(R, A, mu, b, Om, 40, rtol=1e-10, matvec="f32", refine=6, lo="f32")
    assert rc == 0, info
    assert info["precision_used"] == 1
    xt = ot.solve_dense(A, mu, b)
    assert a_err(A, mu, x, xt) < 1e-8
    assert info["relres"] <= 1e-10


def test_repeated_solves_are_bitwise_identical(R):
    """The first solve of a shape autotunes the block product's split count; later solves reuse
    it, and the same inputs give the same iterate bit for bit (fixed summation orders)."""
    import torch
    rbcg, ctx = R
    note("repeat solve d=3000 k=64 f64 and f32")
    P = synth.dense_problem(7, 3000, 1.5, 64, 1e-4)
    op = rbcg.DenseOperator(ctx, to_dev(P["A"]), lo="f32")
    bd, omd = to_dev(P["b"]), to_dev(P["omega"])
    for mv in ("f64", "f32"):
        xs = []
        for _ in range(3):
            x = torch.zeros_like(bd)
            rc, info = rbcg.solve(ctx, [op], [P["mu"]], [bd], [omd], [x],
                                  [rbcg.opts(40, rtol=1e-10, matvec=mv, refine_max=6)], check=False)
            assert rc == 0, info
            xs.append(x.cpu().numpy())
        assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[1], xs[2])


@pytest.mark.parametrize("sweep_tol", [1e-6, 1e-4, 1e-2])
def test_sweep_target_changes_schedule_not_answer(R, sweep_tol):
    """The per-sweep target of low-precision refinement trades sweeps against products per
    sweep; every setting reaches the requested FP64 residual."""
    import torch
    rbcg, ctx = R
    note(f"sweep_tol {sweep_tol}")
    g = np.random.default_rng(6)
    d = 2048
    A = synth.spd_from_spectrum(np.arange(1, d + 1, dtype=float) ** (-1.5), g)
    b = g.standard_normal(d)
    Om = g.standard_normal((64, d))
    op = rbcg.DenseOperator(ctx, to_dev(A), lo="f32")
    bd = to_dev(b)
    x = torch.zeros_like(bd)
    o = rbcg.opts(40, rtol=1e-10, matvec="f32", refine_max=12, sweep_tol=sweep_tol)
    rc, info = rbcg.solve(ctx, [op], [1e-4], [bd], [to_dev(Om)], [x], [o], check=False)
    assert rc == 0, info
    note(f"  sweeps {info[0]['refine_sweeps']} loads {info[0]['matrix_loads']} relres {info[0]['relres']:.1e}")
    assert info[0]["relres"] <= 1e-10
    xt = ot.solve_dense(A, 1e-4, b)
    assert a_err(A, 1e-4, x.cpu().numpy(), xt) < 1e-8


def test_invalid_arguments_rejected_before_device_work(R):
    import torch
    rbcg, ctx = R
    A = to_dev(np.eye(8))
    op = rbcg.DenseOperator(ctx, A)
    b = to_dev(np.ones(8))
    x = torch.zeros_like(b)
    om = to_dev(np.ones((8, 8)))   # k = 8 >= d
    rc, _ = rbcg.solve(ctx, [op], [1e-3], [b], [om], [x], [rbcg.opts(2)], check=False)
    assert rc == -1
    rc, _ = rbcg.solve(ctx, [op], [-1.0], [b], [None], [x], [rbcg.opts(2)], check=False)
    assert rc == -1
    rc, _ = rbcg.solve(ctx, [op], [0.0], [b], [None], [x], [rbcg.opts(0)], check=False)
    assert rc == -1
    rc, _ = rbcg.solve(ctx, [op], [0.0], [b], [None], [x], [rbcg.opts(2, sweep_tol=-1.0)], check=False)
    assert rc == -1
    rc, _ = rbcg.solve(ctx, [op], [0.0], [b], [None], [x], [rbcg.opts(2, sweep_tol=1.0)], check=False)
    assert rc == -1
    # mixed precision without the low-precision copy is unsupported
    rc, _ = rbcg.solve(ctx, [op], [0.0], [b], [None], [x], [rbcg.opts(2, matvec="f32")], check=False)
    assert rc == -7
    assert float(x.abs().sum()) == 0.0
    # sampling: all groups share one block product of at most 256 vectors (9 groups of 32 = 288)
    A64 = to_dev(np.eye(64))
    op64 = rbcg.DenseOperator(ctx, A64)
    Bs = to_dev(np.ones((260, 64)))
    Ys = torch.zeros_like(Bs)
    for fn in (rbcg.sqrt_apply, rbcg.invsqrt_apply):
        rc, _ = fn(ctx, op64, Bs, Ys, rbcg.opts(2, group=32), check=False)
        assert rc == -7
    assert float(Ys.abs().sum()) == 0.0
