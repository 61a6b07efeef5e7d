"""CPU pins of the FP64 oracle against what the paper and the mathematics
fix.  No GPU needed."""
import numpy as np
import pytest

import synth
from oracle import block_cg as ob
from oracle import krylov as ok
from oracle import quadrature as oq
from oracle import truth as ot

from pins import (small_spd, inv_sqrt_identity_gaps, definition_gap, exact_termination_gap, cg_gap, path_gap,
                  sqrt_full_space_gap, quadrature_gap, sampling_definition_gaps, pcg_gap)


# --------------------------------------------------------------- def. BCG / eq. bcg_alg
def test_lanczos_matches_definition():
    """Block-Lanczos + eq. bcg_alg reproduces the def. BCG optimum computed
    over an explicit basis of K_t(A, [b Omega])."""
    assert definition_gap() < 1e-10


def test_path_matches_definition_every_shift():
    """One Krylov space serves every shift (eq. shift_invariance)."""
    assert path_gap() < 1e-10


def test_exact_termination_small():
    """(k+1) t >= d makes K_t the whole space, so the iterate is A_mu^-1 b."""
    assert exact_termination_gap() < 1e-11


def test_k0_is_cg():
    """With Omega empty, block-CG is CG (def. CG vs the Hestenes-Stiefel
    recurrence)."""
    assert cg_gap() < 1e-9


def test_cg_definition_matches_recurrence():
    A, _ = small_spd(50, p=1.0, seed=9)
    b = np.random.default_rng(9).standard_normal(50)
    for t in (1, 3, 6):
        x1 = ok.cg_definition(A, 1e-2, b, t)
        x2 = ok.cg_hestenes_stiefel(A, 1e-2, b, t)
        assert ob.rel_a_err(A, 1e-2, x1, x2) < 1e-10


def test_pcg_definition_matches_textbook_recurrence():
    """def. PCG (optimality over K_t(P^-1 A_mu, P^-1 b)) equals the textbook
    preconditioned CG recurrence for the Nystrom deflation preconditioner
    (eq. precond_def) at every t."""
    assert pcg_gap() < 1e-9


# ------------------------------------------------------------------- C1-shaped problem
@pytest.fixture(scope="module")
def c1():
    return synth.dense_problem(1, 512, 2.0, 16, 1e-3)


def test_c1_exact_termination(c1):
    """C1 (d=512, k=16): 17 * 31 >= 512, so t = 31 products give the exact
    solution; relative A_mu error against a dense Cholesky solve."""
    X, lz = ob.bcg(c1["A"], [c1["mu"]], c1["b"], c1["omega"], 31)
    xt = ot.solve_dense(c1["A"], c1["mu"], c1["b"])
    assert ob.rel_a_err(c1["A"], c1["mu"], X[0], xt) < 1e-12
    assert sum(lz["widths"]) <= 512


def test_c1_monotone_and_beats_cg(c1):
    """The A_mu-norm error is non-increasing in t (nested spaces plus
    optimality, def. BCG) and never worse than CG at equal t (K_t(A,b) is
    inside K_t(A,[b Omega]))."""
    A, mu, b, Om = c1["A"], c1["mu"], c1["b"], c1["omega"]
    xt = ot.solve_dense(A, mu, b)
    errs = []
    for t in range(1, 16):
        X, _ = ob.bcg(A, [mu], b, Om, t)
        errs.append(ob.rel_a_err(A, mu, X[0], xt))
        xc = ok.cg_definition(A, mu, b, t)
        assert errs[-1] <= ob.rel_a_err(A, mu, xc, xt) * (1 + 1e-8) + 1e-13
    e = np.array(errs)
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-8) + 1e-13)
    assert e[-1] < 1e-10


def test_more_augmentation_never_hurts(c1):
    """K_t(A,[b Omega_1]) is inside K_t(A,[b Omega]) when Omega_1 is a subset
    of the columns, so the optimal error can only drop (used in the proof of
    Thm. main_rate)."""
    A, mu, b, Om = c1["A"], c1["mu"], c1["b"], c1["omega"]
    xt = ot.solve_dense(A, mu, b)
    for t in (3, 6):
        e_small = ob.rel_a_err(A, mu, ob.bcg(A, [mu], b, Om[:4], t)[0][0], xt)
        e_big = ob.rel_a_err(A, mu, ob.bcg(A, [mu], b, Om, t)[0][0], xt)
        assert e_big <= e_small * (1 + 1e-8) + 1e-13


def test_lanczos_structure(c1):
    """Q_t orthonormal with Q_t^T b = ||b|| e_1, T_t block tridiagonal with
    bandwidth 2m+1, the block-Lanczos relation A Q_t = Q_t T_t + Q_{t+1} B_t E_t^T,
    and Ritz values inside [lambda_d, lambda_1] (Sec. 3.2)."""
    A, b, Om = c1["A"], c1["b"], c1["omega"]
    t = 8
    X, lz = ob.bcg(A, [0.0], b, Om, t)
    Q, T, m = lz["Q"], lz["T"], 17
    n = Q.shape[1]
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 1e-13 * n
    qb = Q.T @ b
    assert abs(qb[0] - np.linalg.norm(b)) < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(qb[1:]) < 1e-12 * np.linalg.norm(b)
    i, j = np.indices(T.shape)
    band = np.abs(i // m - j // m) <= 1
    assert np.max(np.abs(T[~band])) < 1e-12 * np.max(np.abs(T))
    # the Lanczos relation with the next block from the t-th product
    E = np.zeros((n, lz["widths"][-1]))
    E[n - lz["widths"][-1]:, :] = np.eye(lz["widths"][-1])
    R = lz["AQ"] - Q @ T - lz["Qnext"] @ lz["Bnext"] @ E.T
    assert np.linalg.norm(R) < 1e-12 * np.linalg.norm(lz["AQ"])
    ritz = np.linalg.eigvalsh(T)
    lam = c1["lam"]
    assert ritz.min() >= lam.min() * (1 - 1e-8) and ritz.max() <= lam.max() * (1 + 1e-10)


def test_residual_estimate_matches_true_residual(c1):
    """The a-posteriori residual from the Lanczos relation equals
    ||b - A_mu x_t|| (remark on stopping signals, Sec. 4)."""
    A, mu, b, Om = c1["A"], c1["mu"], c1["b"], c1["omega"]
    for t in (3, 7):
        X, lz = ob.bcg(A, [mu], b, Om, t)
        r_true = np.linalg.norm(b - (A @ X[0] + mu * X[0]))
        r_est = ob.bcg_residual_estimate(lz, mu, np.linalg.norm(b))
        assert abs(r_true - r_est) < 1e-8 * r_true + 1e-13 * np.linalg.norm(b)


def test_thm_main_rate_bound(c1):
    """Thm. main_rate (loose statistical check, one seed): with l = 16
    Gaussian columns, q = 1, p = 2, r = 14, the error is below
    2 exp(-(t-s)/(3 sqrt(kappa_{r+1}(mu)))) for every mu on a grid."""
    A, b, Om, lam = c1["A"], c1["b"], c1["omega"], c1["lam"]
    d, r, p = 512, 14, 2
    tail = np.sum(lam[r:] ** 2) / lam[r] ** 2
    s = min(3 + np.log(d) / 2, 1.5 + 0.25 * np.log(4 + 4 * r / (p - 1) * tail))
    mus = [0.0, 1e-6, 1e-3, 1e-1]
    for t in (int(np.ceil(s)) + 2, 12, 20):
        X, _ = ob.bcg(A, mus, b, Om, t)
        for i, mu in enumerate(mus):
            xt = ot.solve_dense(A, mu, b) if mu > 0 else np.linalg.solve(A, b)
            kap = (lam[r] + mu) / (lam[-1] + mu)
            bound = 2 * np.exp(-(t - s) / (3 * np.sqrt(kap)))
            assert ob.rel_a_err(A, mu, X[i], xt) <= bound * (1 + 1e-6) + 1e-10


# -------------------------------------------------------------- Thm. main and Nystrom
@pytest.fixture(scope="module")
def nys_problem():
    A, lam = small_spd(160, p=2.0, seed=21)
    g = np.random.default_rng(22)
    return {"A": A, "lam": lam, "b": g.standard_normal(160), "omega": g.standard_normal((8, 160))}


@pytest.mark.parametrize("s", [1, 3])
def test_thm_main_block_cg_beats_nystrom_pcg(nys_problem, s):
    """Thm. main: err(bcg_t) <= err(pcg_{t-s}) for the Nystrom deflation
    preconditioner built from the same Omega, for theta = the smallest
    Nystrom eigenvalue (the experiments' rule) and other theta."""
    A, b, Om = nys_problem["A"], nys_problem["b"], nys_problem["omega"]
    U, D = ok.nystrom(A, Om, s)
    for mu in (1e-4, 1e-2):
        xt = ot.solve_dense(A, mu, b)
        for theta in (D.min(), 10 * D.min(), 0.1 * D.min()):
            Pinv = ok.deflation_pinv(U, D, theta, mu)
            for t in (s + 1, s + 3, s + 6):
                e_b = ob.rel_a_err(A, mu, ob.bcg(A, [mu], b, Om, t)[0][0], xt)
                e_p = ob.rel_a_err(A, mu, ok.pcg_definition(A, mu, b, Pinv, t - s), xt)
                assert e_b <= e_p * (1 + 1e-7) + 1e-12


def test_nystrom_properties(nys_problem):
    """A<K> is below A in the Loewner order, and Prop. condno_perturb bounds
    the preconditioned condition number for any theta."""
    A, lam, Om = nys_problem["A"], nys_problem["lam"], nys_problem["omega"]
    for s in (1, 2):
        U, D = ok.nystrom(A, Om, s)
        An = ok.nystrom_matrix(U, D)
        assert np.linalg.eigvalsh(A - An).min() > -1e-12 * lam[0]
        err = np.linalg.norm(A - An, 2)
        for mu in (1e-4, 1e-2):
            for theta in (D.min(), lam[-1], 3 * D.min()):
                kap = ok.condition_number_preconditioned(A, mu, ok.deflation_pinv(U, D, theta, mu))
                bound = (theta + mu + err) * (1 / (theta + mu) + 1 / (lam[-1] + mu))
                assert kap <= bound * (1 + 1e-8)


def test_nystrom_range_in_krylov(nys_problem):
    """range(A<K_s>) lies in K_{s+1}(A, Omega) (footnote to the remark after
    Thm. main), so P^-1 = I + X with range(X) in that space."""
    A, Om = nys_problem["A"], nys_problem["omega"]
    s = 2
    U, _ = ok.nystrom(A, Om, s)
    V = ob.krylov_basis_explicit(lambda X: A @ X, Om.T, s + 1)
    assert np.linalg.norm(U - V @ (V.T @ U)) < 1e-8


# --------------------------------------------------------------------------- sampling
def test_sqrt_full_space_exact():
    """m t >= d: block-Lanczos square root equals A^(1/2) B (def. blansq)."""
    assert sqrt_full_space_gap() < 1e-10


def test_inv_sqrt_full_space_exact():
    A, _ = small_spd(40, p=1.0, seed=7)
    B = np.random.default_rng(8).standard_normal((8, 40))
    Y, _ = ob.inv_sqrt_apply_exact(A, B, 5)
    Yt = ot.inv_sqrt_eig(A, B)
    assert np.max(np.linalg.norm(Y - Yt, axis=1) / np.linalg.norm(Yt, axis=1)) < 1e-9


def test_inv_sqrt_is_A_inverse_of_sqrt_iterate():
    """Sec. 5.1 after def. blanisq: bisq_t = A^-1 bsq_t at every t (here m t < d)
    and the error bound that follows from it."""
    gap, ratio = inv_sqrt_identity_gaps()
    assert gap <= 1e-12
    assert ratio <= 1.0 + 1e-10


def test_sampling_iterates_match_definition_outside_full_space():
    """m t < d: the square-root and inverse-square-root iterates equal the
    z-integral of the shifted block-CG iterates (def. blansq, def. blanisq)
    over an explicit basis of K_t(A, B), integrated numerically."""
    gs, gi = sampling_definition_gaps()
    assert gs < 1e-10 and gi < 1e-10


def test_sqrt_quadrature_matches_closed_form():
    """The quadrature form of the block-Lanczos square root agrees with the
    closed form A Q T^-1/2 Q^T B to the rule's accuracy, using Ritz bounds."""
    A, _ = small_spd(300, p=1.5, seed=11)
    B = np.random.default_rng(12).standard_normal((8, 300))
    Ye, lz = ob.sqrt_apply_exact(A, B, 6)
    ritz = np.linalg.eigvalsh(lz["T"])
    s, w = oq.sqrt_rule(ritz[0], ritz[-1], 32)
    Yq, _ = ob.sqrt_apply_quadrature(A, B, 6, s, w, lz=lz)
    assert np.max(np.linalg.norm(Yq - Ye, axis=1) / np.linalg.norm(Ye, axis=1)) < 1e-11


def test_quadrature_rule_scalar_accuracy():
    """sum_j w_j lam/(lam+s_j) = sqrt(lam) across [m, M] (eq. sqrt_rational)."""
    assert quadrature_gap() < 1e-11
    assert quadrature_gap(1e-3, 1.0, 16) < 1e-12


def test_quadrature_reproduces_elliptic_identity():
    """eq. ellipticK_eval: the same rule applied to ((l1+z^2)(ld+z^2))^-1/2
    gives K(1 - l1/ld)/sqrt(ld); the numeric integral agrees too."""
    l1, ld = 244.0, 3.6e-3
    s, w = oq.sqrt_rule(ld, l1, 48)
    z2 = s
    # the rule integrates (2/pi) int g(z) dz with weights w for g = lam/(lam+z^2);
    # for a general g the weight of node j is w_j, the integrand g(z_j)
    approx = np.pi / 2 * np.sum(w / np.sqrt((l1 + z2) * (ld + z2)))
    exact = oq.elliptic_integral_eval(l1, ld)
    assert abs(approx - exact) < 1e-9 * exact
    assert abs(oq.elliptic_integral_numeric(l1, ld) - exact) < 1e-12 * exact


@pytest.mark.parametrize("x", [1.0001, 2.0, 1e3, 1e8])
def test_lemma_elliptic_k_bound(x):
    """Lemma elliptic_k_bd: (2/pi) sqrt(x) K(1-x) <= 5/(4 pi) log(16x) <= log(16x)/2."""
    a, b, c = oq.lemma_elliptic_sides(x)
    assert a <= b * (1 + 1e-14) and b <= c


# ------------------------------------------------------------------------------ ridge
def test_ridge_truths_agree():
    """The SVD route, the Gram eigendecomposition route and a dense Cholesky
    on Z^T Z + mu I agree on the ridge path (eq. ridge_regression)."""
    g = np.random.default_rng(31)
    Z = (g.standard_normal((300, 40)) * np.exp(-np.arange(1, 41) / 10)).astype(np.float32)
    f = g.standard_normal(300)
    Z64 = Z.astype(np.float64)
    b = Z64.T @ f
    mus = [1e-4, 1e-2, 1.0]
    X1 = ot.ridge_path_svd(Z, f, mus)
    X2 = ot.ridge_path_eig_gram(Z, b, mus)
    X4 = ot.ridge_path_qr_svd(Z, f, mus)
    X5 = ot.ridge_path_qr_svd(Z, f, mus, rows_per_block=70)
    for i, mu in enumerate(mus):
        x3 = ot.solve_dense(Z64.T @ Z64, mu, b)
        assert np.linalg.norm(X1[i] - x3) < 1e-8 * np.linalg.norm(x3)
        assert np.linalg.norm(X2[i] - x3) < 1e-8 * np.linalg.norm(x3)
        assert np.linalg.norm(X4[i] - x3) < 1e-8 * np.linalg.norm(x3)
        assert np.linalg.norm(X5[i] - x3) < 1e-8 * np.linalg.norm(x3)


def test_ridge_block_cg_path_exact():
    """With the Gram operator and m t >= d the whole path is exact."""
    g = np.random.default_rng(32)
    Z = (g.standard_normal((500, 48)) * np.exp(-np.arange(1, 49) / 16)).astype(np.float32)
    f = g.standard_normal(500)
    b = Z.astype(np.float64).T @ f
    Om = g.standard_normal((7, 48))
    mus = np.logspace(-6, 0, 7)
    X, _ = ob.bcg(ob.gram_operator(Z), mus, b, Om, 6)
    Xt = ot.ridge_path_svd(Z, f, mus)
    A = Z.astype(np.float64).T @ Z.astype(np.float64)
    for i, mu in enumerate(mus):
        assert ob.rel_a_err(A, mu, X[i], Xt[i]) < 1e-7


# ------------------------------------------------------------------------- refinement
def test_refinement_converges_to_dense_solution():
    A, _ = small_spd(120, p=1.5, seed=41)
    g = np.random.default_rng(42)
    b = g.standard_normal(120)
    Om = g.standard_normal((6, 120))
    x = ob.bcg_refined(A, 1e-4, b, Om, 12, 6)
    xt = ot.solve_dense(A, 1e-4, b)
    assert ob.rel_a_err(A, 1e-4, x, xt) < 1e-12


def test_deflation_of_dependent_columns():
    """Duplicate Omega columns and an Omega column equal to b are dropped as
    rank-deficient directions; the iterate is unchanged."""
    A, _ = small_spd(50, p=1.0, seed=51)
    g = np.random.default_rng(52)
    b = g.standard_normal(50)
    Om = g.standard_normal((3, 50))
    Om_dup = np.vstack([Om, Om[:1], b[None, :]])
    for t in (2, 4):
        x1 = ob.bcg(A, [1e-3], b, Om, t)[0][0]
        x2, lz = ob.bcg(A, [1e-3], b, Om_dup, t)
        assert lz["widths"][0] == 4
        assert ob.rel_a_err(A, 1e-3, x2[0], x1) < 1e-9
