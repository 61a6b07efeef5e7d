"""GPU parity of rbcg_path (regularization path, dense and Gram operators) and
rbcg_sqrt_apply (block-Lanczos square root) against the FP64 CPU oracle, all
through the C ABI.

Tolerances: path iterates vs the oracle's bcg_t at every shift to
max(1e-12, 0.1 kappa(A_mu) u) in the A_mu-norm (plain FP64); mixed BF16 Gram
products with FP64 refinement vs the dense ridge solution to 1e-8.  The
square root is compared with the oracle's closed form A Q T^{-1/2} Q^T B; the
GPU integrates with a 32-node conformal-map rule on its own Ritz interval,
whose error is below 1e-10 for these spectra, so the bound is 1e-9 relative
per sample.  The inverse square root (rbcg_invsqrt_apply) uses the same rule,
whose relative error per Ritz value is the same for l^{-1/2} as for l^{1/2}
(the two sums differ by the factor l), and is compared with the oracle's
Q T^{-1/2} Q^T B to the same bound; its spectra are kept at kappa <= 1e4 so
that rounding in the two Lanczos runs, which the inverse amplifies at the
small end of the spectrum, stays well below it.
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
    return rbcg, rbcg.Context()


def _path(R, op, b, Om, mus, t, **kw):
    import torch
    rbcg, ctx = R
    bd = to_dev(b)
    om = to_dev(Om) if Om is not None and len(Om) else None
    X = torch.zeros((len(mus), b.shape[0]), dtype=torch.float64, device="cuda")
    rc, info = rbcg.path(ctx, op, bd, om, list(mus), X, rbcg.opts(t, **kw), check=False)
    torch.cuda.synchronize()
    return rc, info, X.cpu().numpy()


@pytest.mark.parametrize("d,k,t,L", [(400, 15, 6, 8), (333, 20, 4, 5), (256, 31, 9, 16)])
def test_dense_path_matches_oracle_every_shift(R, d, k, t, L):
    """One Krylov space, L shifts (eq. bcg_alg): every shift equals the
    oracle's iterate from the same space."""
    rbcg, ctx = R
    note(f"dense path d={d} k={k} t={t} L={L}")
    g = np.random.default_rng(d)
    lam = np.arange(1, d + 1, dtype=float) ** (-1.5)
    A = synth.spd_from_spectrum(lam, g)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    mus = np.logspace(-5, 0, L)
    op = rbcg.DenseOperator(ctx, to_dev(A))
    rc, info, X = _path(R, op, b, Om, mus, t)
    assert rc == 0, info
    Xo, _ = ob.bcg(A, mus, b, Om, t)
    for i, mu in enumerate(mus):
        kappa = (lam[0] + mu) / (lam[-1] + mu)
        assert a_err(A, mu, X[i], Xo[i]) < fp64_bound(kappa), (i, mu)


@pytest.fixture(scope="module")
def ridge_small():
    """A scaled-down ridge problem with the same construction as the
    200000 x 4096 workload: Z = G diag(exp(-j/decay)), FP32."""
    return synth.ridge_problem(3, 6000, 384, 63, decay=40.0, L=12)


def test_gram_path_fp64_exact_termination(R, ridge_small):
    """Gram operator Z^T (Z X) with FP64 arithmetic on the FP32 values of Z;
    64 * 6 >= 384 so every shift is exact: compare with the SVD ridge path."""
    rbcg, ctx = R
    P = ridge_small
    note("gram path fp64 exact")
    Zd = to_dev(P["Z"])
    op = rbcg.GramOperator(ctx, Zd, lo="f64")
    rc, info, X = _path(R, op, P["b"], P["omega"], P["mus"], 6)
    assert rc == 0, info
    Z64 = P["Z"].astype(np.float64)
    A = Z64.T @ Z64
    Xt = ot.ridge_path_svd(P["Z"], P["f"], P["mus"])
    for i, mu in enumerate(P["mus"]):
        lam = np.linalg.eigvalsh(A)
        kappa = (lam[-1] + mu) / (lam[0] + mu)
        assert a_err(A, mu, X[i], Xt[i]) < max(1e-11, 1e-15 * kappa), (i, mu)


def test_gram_path_fp64_iterates_match_oracle(R, ridge_small):
    rbcg, ctx = R
    P = ridge_small
    note("gram path fp64 t=3")
    op = rbcg.GramOperator(ctx, to_dev(P["Z"]), lo="f64")
    rc, info, X = _path(R, op, P["b"], P["omega"], P["mus"], 3)
    assert rc == 0, info
    Xo, _ = ob.bcg(ob.gram_operator(P["Z"]), P["mus"], P["b"], P["omega"], 3)
    Z64 = P["Z"].astype(np.float64)
    A = Z64.T @ Z64
    for i, mu in enumerate(P["mus"]):
        assert a_err(A, mu, X[i], Xo[i]) < 1e-10, (i, mu)


def test_gram_path_bf16_refined_reaches_fp64_answer(R, ridge_small):
    """BF16 Z and Z^T copies on MFMA (three-part BF16 vectors) with FP64
    refinement: every shift within 1e-8 of the dense ridge solution.  Here
    t_max m >= d, so the first space is built out to R^d and the refinement
    steps reuse it (one FP64 residual product per step, no new space)."""
    rbcg, ctx = R
    P = ridge_small
    note("gram path bf16 refine")
    op = rbcg.GramOperator(ctx, to_dev(P["Z"]), lo="bf16")
    rc, info, X = _path(R, op, P["b"], P["omega"], P["mus"], 8, rtol=1e-12, matvec="bf16", refine_max=12)
    assert rc == 0, info
    note(f"  loads {info[0]['matrix_loads']} sweeps/steps {info[0]['refine_sweeps']} iters {info[0]['iters']}")
    # the first space spans R^d after ceil(384 / 64) = 6 products; the rest are recycled steps and
    # at most a few fresh sweeps
    assert info[0]["matrix_loads"] <= 6 + 1 + 12 + 2 * 6, info[0]
    Z64 = P["Z"].astype(np.float64)
    A = Z64.T @ Z64
    Xt = ot.ridge_path_svd(P["Z"], P["f"], P["mus"])
    for i, mu in enumerate(P["mus"]):
        assert a_err(A, mu, X[i], Xt[i]) < 1e-8, (i, mu, info[i])
    assert all(inf["precision_used"] == 2 for inf in info)


def test_dense_path_fp32_refined_partial_spaces(R):
    """FP32 products with FP64 refinement where one Krylov space cannot span
    R^d (t_max m = 384 < d = 600): each refinement sweep builds a fresh space
    on [R Omega]; every shift reaches rtol and lies within 1e-8 of the dense
    solve in A_mu-norm."""
    rbcg, ctx = R
    P = synth.dense_problem(7, 600, 1.5, 31, 1e-3)
    A, b = P["A"], P["b"]
    mus = [float(v) for v in np.logspace(-4, -1, 8)]
    note("dense path f32 refine d=600 k=31 t=12 L=8")
    op = rbcg.DenseOperator(ctx, to_dev(A), lo="f32")
    rc, info, X = _path(R, op, b, P["omega"], mus, 12, rtol=1e-11, matvec="f32", refine_max=20)
    assert rc == 0, info
    note(f"  loads {info[0]['matrix_loads']} sweeps {info[0]['refine_sweeps']}")
    assert info[0]["refine_sweeps"] >= 2
    for i, mu in enumerate(mus):
        xt = np.linalg.solve(A + mu * np.eye(A.shape[0]), b)
        assert a_err(A, mu, X[i], xt) < 1e-8, (i, mu, info[i])
        assert info[i]["relres"] <= 1e-11


def _sqrt(R, op, B, t, nquad=32, group=32, matvec="f64", inverse=False):
    import torch
    rbcg, ctx = R
    Bd = to_dev(B)
    Y = torch.zeros_like(Bd)
    fn = rbcg.invsqrt_apply if inverse else rbcg.sqrt_apply
    rc, info = fn(ctx, op, Bd, Y, rbcg.opts(t, nquad=nquad, group=group, matvec=matvec), check=False)
    torch.cuda.synchronize()
    return rc, info, Y.cpu().numpy()


@pytest.fixture(scope="module")
def rbf_small():
    return synth.rbf_problem(4, 1024, 64, ell=0.2)


def test_sqrt_matches_oracle_closed_form(R, rbf_small):
    """Two groups of 32 samples, one shared pass over A per step; each group
    equals the oracle's block-Lanczos square root of its own block."""
    rbcg, ctx = R
    P = rbf_small
    note("sqrt rbf d=1024 t=8")
    A, B = P["A"], P["B"]
    op = rbcg.DenseOperator(ctx, to_dev(A))
    t = 8
    rc, info, Y = _sqrt(R, op, B, t)
    assert rc == 0, info
    for g in range(2):
        Yo, _ = ob.sqrt_apply_exact(A, B[32 * g:32 * (g + 1)], t)
        Yg = Y[32 * g:32 * (g + 1)]
        rel = np.linalg.norm(Yg - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
        assert rel.max() < 1e-9, rel.max()


def test_sqrt_fp32_products_pinned_on_rounded_operands(R):
    """FP32 block products (A and each block rounded to FP32, FP32 MFMA
    accumulation) against the oracle run on the same rounded operands with
    exact accumulation.  What separates the two is the kernel's FP32
    accumulation; its size on this operator is measured through
    rbcg_op_apply (largest column-relative error eps of one block product),
    and the bound is four times the change the oracle shows when each of its
    products is perturbed by eps.  RBF kernel matrix on 2000 points (ragged
    last tile) with a 1e-2 nugget, kappa ~ 3e3; two groups of 32."""
    import torch
    rbcg, ctx = R
    P = synth.rbf_problem(6, 2000, 64, ell=0.1, nugget=1e-2)
    A, B = P["A"], P["B"]
    note("sqrt fp32 rbf d=2000 nugget 1e-2 t=10")
    op = rbcg.DenseOperator(ctx, to_dev(A), lo="f32")
    t = 10
    rc, info, Y = _sqrt(R, op, B, t, matvec="f32")
    assert rc == 0, info
    A32 = A.astype(np.float32).astype(np.float64)

    def op32(X):
        return A32 @ np.asarray(X).astype(np.float32).astype(np.float64)

    # accumulation error of the FP32 kernel on this operator, one 64-vector block
    X = synth.rng(31, 0).standard_normal((64, A.shape[0]))
    W = torch.zeros((64, A.shape[0]), dtype=torch.float64, device="cuda")
    rbcg.op_apply(ctx, op, to_dev(X), W, "f32")
    Wr = op32(X.T).T
    eps = float((np.linalg.norm(W.cpu().numpy() - Wr, axis=1) / np.linalg.norm(Wr, axis=1)).max())
    g = np.random.default_rng(77)

    def op32_perturbed(X):
        Wp = op32(X)
        G = g.standard_normal(Wp.shape)
        return Wp + eps * G * (np.linalg.norm(Wp, axis=0) / np.linalg.norm(G, axis=0))

    def rel(Ya, Yb):
        return float((np.linalg.norm(Ya - Yb, axis=1) / np.linalg.norm(Yb, axis=1)).max())

    for grp in range(2):
        Bg = B[32 * grp:32 * grp + 32]
        Yr, _ = ob.sqrt_apply_exact(op32, Bg, t)
        Yp, _ = ob.sqrt_apply_exact(op32_perturbed, Bg, t)
        Yo, _ = ob.sqrt_apply_exact(A, Bg, t)
        sens = rel(Yp, Yr)
        e = rel(Y[32 * grp:32 * grp + 32], Yr)
        note(f"group {grp}: product eps {eps:.1e}; FP32 GPU vs oracle on rounded operands {e:.2e} "
             f"(bound 4 x {sens:.2e}); vs FP64 oracle {rel(Y[32 * grp:32 * grp + 32], Yo):.2e}")
        assert e <= 4.0 * sens


def test_sqrt_ragged_last_group(R):
    """40 samples in groups of 16: the last group has 8 samples (its block is
    zero padded and the padding deflates); every group equals the oracle's
    square root over its own block."""
    rbcg, ctx = R
    note("sqrt ragged groups")
    g = np.random.default_rng(77)
    d = 200
    A = synth.spd_from_spectrum(np.linspace(1.0, 50.0, d) ** 2, g)
    B = g.standard_normal((40, d))
    op = rbcg.DenseOperator(ctx, to_dev(A))
    t = 5
    rc, info, Y = _sqrt(R, op, B, t, group=16)
    assert rc == 0, info
    for g0, g1 in [(0, 16), (16, 32), (32, 40)]:
        Yo, _ = ob.sqrt_apply_exact(A, B[g0:g1], t)
        rel = np.linalg.norm(Y[g0:g1] - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
        assert rel.max() < 1e-9, (g0, rel.max())


def test_sqrt_full_space_equals_eigh(R):
    """m t >= d: the block-Lanczos square root is A^{1/2} B exactly."""
    rbcg, ctx = R
    note("sqrt full space")
    g = np.random.default_rng(78)
    d = 96
    A = synth.spd_from_spectrum(np.linspace(1.0, 50.0, d), g)
    B = g.standard_normal((48, d))
    op = rbcg.DenseOperator(ctx, to_dev(A))
    rc, info, Y = _sqrt(R, op, B, 7, group=16)
    assert rc == 0, info
    Yt = ot.sqrt_eig(A, B)
    rel = np.linalg.norm(Y - Yt, axis=1) / np.linalg.norm(Yt, axis=1)
    assert rel.max() < 1e-9, rel.max()


def test_invsqrt_matches_oracle_closed_form(R):
    """Inverse square root (def. blanisq), two groups of 32 samples sharing each
    pass over A: each group equals the oracle's Q T^{-1/2} Q^T B of its block."""
    rbcg, ctx = R
    note("invsqrt rbf d=1024 t=8")
    P = synth.rbf_problem(4, 1024, 64, ell=0.2, nugget=1e-2)
    A, B = P["A"], P["B"]
    op = rbcg.DenseOperator(ctx, to_dev(A))
    t = 8
    rc, info, Y = _sqrt(R, op, B, t, inverse=True)
    assert rc == 0, info
    for g in range(2):
        Yo, _ = ob.inv_sqrt_apply_exact(A, B[32 * g:32 * (g + 1)], t)
        Yg = Y[32 * g:32 * (g + 1)]
        rel = np.linalg.norm(Yg - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
        assert rel.max() < 1e-9, rel.max()


def test_invsqrt_ragged_last_group(R):
    """40 samples in groups of 16 (the last group padded to 16, the padding
    deflates): every group equals the oracle's inverse square root."""
    rbcg, ctx = R
    note("invsqrt ragged groups")
    g = np.random.default_rng(79)
    d = 200
    A = synth.spd_from_spectrum(np.linspace(1.0, 50.0, d) ** 2, g)
    B = g.standard_normal((40, d))
    op = rbcg.DenseOperator(ctx, to_dev(A))
    t = 5
    rc, info, Y = _sqrt(R, op, B, t, group=16, inverse=True)
    assert rc == 0, info
    for g0, g1 in [(0, 16), (16, 32), (32, 40)]:
        Yo, _ = ob.inv_sqrt_apply_exact(A, B[g0:g1], t)
        rel = np.linalg.norm(Y[g0:g1] - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
        assert rel.max() < 1e-9, (g0, rel.max())


def test_invsqrt_full_space_equals_eigh(R):
    """m t >= d: the block-Lanczos inverse square root is A^{-1/2} B exactly,
    and applying the square root to it gives B back."""
    rbcg, ctx = R
    note("invsqrt full space")
    g = np.random.default_rng(80)
    d = 96
    A = synth.spd_from_spectrum(np.linspace(1.0, 50.0, d), g)
    B = g.standard_normal((48, d))
    op = rbcg.DenseOperator(ctx, to_dev(A))
    rc, info, Y = _sqrt(R, op, B, 7, group=16, inverse=True)
    assert rc == 0, info
    Yt = ot.inv_sqrt_eig(A, B)
    rel = np.linalg.norm(Y - Yt, axis=1) / np.linalg.norm(Yt, axis=1)
    assert rel.max() < 1e-9, rel.max()
    rc, info, Z = _sqrt(R, op, Y, 7, group=16)
    assert rc == 0, info
    rel = np.linalg.norm(Z - B, axis=1) / np.linalg.norm(B, axis=1)
    assert rel.max() < 1e-9, rel.max()


def test_sqrt_and_invsqrt_chunked_product(R):
    """160 samples in 5 groups of 32: the fused block product of 160 vectors runs
    as two column chunks of 80; every group of both the square root and the
    inverse square root equals the oracle's closed form of its own block."""
    rbcg, ctx = R
    note("sqrt + invsqrt, 160 fused vectors (two chunks)")
    g = np.random.default_rng(81)
    d = 600
    A = synth.spd_from_spectrum(np.linspace(1.0, 50.0, d), g)
    B = g.standard_normal((160, d))
    op = rbcg.DenseOperator(ctx, to_dev(A))
    t = 4
    for inverse, ref in ((False, ob.sqrt_apply_exact), (True, ob.inv_sqrt_apply_exact)):
        rc, info, Y = _sqrt(R, op, B, t, inverse=inverse)
        assert rc == 0, info
        for g0 in range(0, 160, 32):
            Yo, _ = ref(A, B[g0:g0 + 32], t)
            rel = np.linalg.norm(Y[g0:g0 + 32] - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
            assert rel.max() < 1e-9, (inverse, g0, rel.max())
