"""Pin checks for the oracle, written as functions that return a residual so
that the planted-mistake tests can show each pin rejects a wrong oracle.

Each function cites the statement of the paper (or the textbook fact) it
pins against.  None of them re-types the oracle's own formula: they compare
against an independent route (an explicit Krylov basis, a dense
factorization, a textbook recurrence, a theorem's inequality).
"""
from __future__ import annotations

import numpy as np

import synth
from oracle import block_cg as ob
from oracle import krylov as ok
from oracle import quadrature as oq
from oracle import truth as ot


def small_spd(d, p=2.0, seed=0, scale=1.0):
    g = np.random.default_rng(seed)
    lam = scale * np.arange(1, d + 1, dtype=float) ** (-p)
    Q = synth.orthogonal(d, g)
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), lam


def definition_gap(d=36, k=2, ts=(1, 2, 3, 4), mu=1e-2, seed=1):
    """max over t of the relative A_mu error between the block-Lanczos
    oracle and the def. BCG Galerkin solution over an explicit basis."""
    A, _ = small_spd(d, p=1.0, seed=seed)
    g = np.random.default_rng(seed + 100)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    worst = 0.0
    for t in ts:
        X, _ = ob.bcg(A, [mu], b, Om, t)
        xd = ob.bcg_definition(A, mu, b, Om, t)
        worst = max(worst, ob.rel_a_err(A, mu, X[0], xd))
    return worst


def exact_termination_gap(d=60, k=5, t=10, mu=1e-3, seed=2):
    """(k+1) t >= d: block-CG is exact; relative A_mu error against a dense
    Cholesky solve."""
    A, _ = small_spd(d, p=2.0, seed=seed)
    g = np.random.default_rng(seed + 100)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    X, _ = ob.bcg(A, [mu], b, Om, t)
    return ob.rel_a_err(A, mu, X[0], ot.solve_dense(A, mu, b))


def cg_gap(d=80, t_max=10, mu=1e-2, seed=3):
    """k = 0: block-CG reduces to CG; compare with the textbook
    Hestenes-Stiefel recurrence at every t."""
    A, _ = small_spd(d, p=1.0, seed=seed)
    b = np.random.default_rng(seed + 100).standard_normal(d)
    worst = 0.0
    for t in range(1, t_max + 1):
        X, _ = ob.bcg(A, [mu], b, None, t)
        xc = ok.cg_hestenes_stiefel(A, mu, b, t)
        worst = max(worst, ob.rel_a_err(A, mu, X[0], xc))
    return worst


def path_gap(d=40, k=3, t=3, seed=4):
    """Shift invariance: the path from one Krylov space equals the
    definition-tier solution at every shift (eq. shift_invariance, eq.
    bcg_alg)."""
    A, _ = small_spd(d, p=1.0, seed=seed)
    g = np.random.default_rng(seed + 100)
    b = g.standard_normal(d)
    Om = g.standard_normal((k, d))
    mus = [0.0, 1e-3, 1e-1, 1.0]
    X, _ = ob.bcg(A, mus, b, Om, t)
    return max(ob.rel_a_err(A, mu, X[i], ob.bcg_definition(A, mu, b, Om, t)) for i, mu in enumerate(mus))


def sqrt_full_space_gap(d=48, m=8, t=6, seed=5):
    """m t >= d: the block-Lanczos square root is exact; compare with
    A^(1/2) B by eigendecomposition (def. blansq)."""
    A, _ = small_spd(d, p=1.0, seed=seed)
    B = np.random.default_rng(seed + 100).standard_normal((m, d))
    Y, _ = ob.sqrt_apply_exact(A, B, t)
    Yt = ot.sqrt_eig(A, B)
    return float(np.max(np.linalg.norm(Y - Yt, axis=1) / np.linalg.norm(Yt, axis=1)))


def quadrature_gap(m=1e-6, M=244.0, N=32):
    """Scalar accuracy of the square-root rule on a log grid of [m, M]."""
    s, w = oq.sqrt_rule(m, M, N)
    lam = np.logspace(np.log10(m), np.log10(M), 301)
    return float(np.max(np.abs(oq.apply_rule_scalar(lam, s, w) - np.sqrt(lam)) / np.sqrt(lam)))


def inv_sqrt_identity_gaps(d=60, m=8, ts=(1, 2, 3), seed=21):
    """Sec. 5.1 after def. blanisq: bisq_t = A^-1 bsq_t at every t, hence
    ||A^-1/2 B - bisq_t|| <= ||A^-1|| ||A^1/2 B - bsq_t||.  Returns the largest
    relative identity gap ||bisq_t A - bsq_t|| / ||bsq_t|| and the largest ratio of
    the error to its bound, over t (m t < d, so no iterate is exact)."""
    from oracle import truth as ot
    A, lam = small_spd(d, p=1.0, seed=seed)
    B = np.random.default_rng(seed + 1).standard_normal((m, d))
    gap = ratio = 0.0
    for t in ts:
        Ys, _ = ob.sqrt_apply_exact(A, B, t)
        Yi, _ = ob.inv_sqrt_apply_exact(A, B, t)
        gap = max(gap, np.linalg.norm(Yi @ A - Ys) / np.linalg.norm(Ys))
        err_i = np.linalg.norm(ot.inv_sqrt_eig(A, B) - Yi)
        err_s = np.linalg.norm(ot.sqrt_eig(A, B) - Ys)
        ratio = max(ratio, err_i / ((1.0 / lam.min()) * err_s))
    return gap, ratio


def _z_integral(H, R, lead=None):
    """(2/pi) int_0^inf lead (H + z^2 I)^-1 R dz by adaptive quadrature in
    phi = arctan z (dz = (1 + z^2) dphi, finite integrand on [0, pi/2]).
    This is the integral that defines the block-Lanczos square root and its
    inverse (def. blansq, def. blanisq), evaluated numerically rather than
    through a matrix power."""
    from scipy.integrate import quad_vec
    n = H.shape[0]
    eye = np.eye(n)

    def f(phi):
        z2 = np.tan(phi) ** 2
        Y = np.linalg.solve(H + z2 * eye, R) * (1.0 + z2)
        return Y if lead is None else lead @ Y
    val, _ = quad_vec(f, 0.0, np.pi / 2, epsabs=1e-14, epsrel=1e-12, limit=400)
    return (2.0 / np.pi) * val


def sampling_definition_gaps(d=60, m=4, ts=(1, 2, 3, 5), seed=31):
    """Sampling iterates outside the full space (m t < d) against their
    definition.  For the samples B (m x d), every shifted block-CG iterate
    bcg_t(z^2) of def. blansq is the Galerkin solution over K_t(A, B^T)
    (def. BCG with the other samples as augmentation), i.e.
    V (V^T A V + z^2 I)^-1 V^T b_i for any orthonormal basis V of that space.
    Here V comes from the explicit blocks [B, AB, ..., A^(t-1) B] (no
    block-Lanczos) and the z-integral is done by adaptive quadrature (no
    matrix square root).  Returns the largest relative gaps (square root,
    inverse square root) over t and samples."""
    A, _ = small_spd(d, p=1.0, seed=seed)
    B = np.random.default_rng(seed + 1).standard_normal((m, d))
    gs = gi = 0.0
    for t in ts:
        assert m * t < d
        V = ob.krylov_basis_explicit(lambda X: A @ X, B.T, t)
        H = V.T @ A @ V
        H = 0.5 * (H + H.T)
        R = V.T @ B.T
        Ys_def = _z_integral(H, R, lead=A @ V).T
        Yi_def = (V @ _z_integral(H, R)).T
        Ys, _ = ob.sqrt_apply_exact(A, B, t)
        Yi, _ = ob.inv_sqrt_apply_exact(A, B, t)
        gs = max(gs, float(np.max(np.linalg.norm(Ys - Ys_def, axis=1) / np.linalg.norm(Ys_def, axis=1))))
        gi = max(gi, float(np.max(np.linalg.norm(Yi - Yi_def, axis=1) / np.linalg.norm(Yi_def, axis=1))))
    return gs, gi


def pcg_textbook(A, mu, b, Pinv, t):
    """Textbook preconditioned conjugate gradients for A_mu x = b with the
    SPD preconditioner inverse Pinv, from x_0 = 0, t steps.  In exact
    arithmetic its t-th iterate minimises the A_mu-norm error over
    K_t(P^-1 A_mu, P^-1 b), i.e. it is pcg_t of def. PCG (Sec. 2.1)."""
    x = np.zeros_like(b, dtype=np.float64)
    r = np.array(b, dtype=np.float64, copy=True)
    z = Pinv @ r
    p = z.copy()
    rz = r @ z
    for _ in range(t):
        Ap = A @ p + mu * p
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = Pinv @ r
        rz_new = r @ z
        if rz_new <= 0.0:
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def pcg_gap(d=120, ell=6, s=2, t_max=8, seed=41):
    """pcg_definition (Galerkin over an explicit basis of the preconditioned
    Krylov space) against the textbook PCG recurrence at every t, with the
    Nystrom deflation preconditioner of eq. precond_def built from a Gaussian
    Omega (theta = the smallest Nystrom eigenvalue) and for two shifts."""
    A, _ = small_spd(d, p=2.0, seed=seed)
    g = np.random.default_rng(seed + 1)
    b = g.standard_normal(d)
    Om = g.standard_normal((ell, d))
    U, D = ok.nystrom(A, Om, s)
    worst = 0.0
    for mu in (1e-3, 1e-1):
        Pinv = ok.deflation_pinv(U, D, D.min(), mu)
        for t in range(1, t_max + 1):
            x_def = ok.pcg_definition(A, mu, b, Pinv, t)
            x_rec = pcg_textbook(A, mu, b, Pinv, t)
            worst = max(worst, ob.rel_a_err(A, mu, x_def, x_rec))
    return worst
