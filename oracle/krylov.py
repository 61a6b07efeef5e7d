"""Single-vector Krylov comparison methods (float64, CPU).  Test
infrastructure only: used to pin the block-CG oracle against the paper's
comparisons, never by the GPU library.

Passages followed:
  * CG by optimality                              Sec. 2.1, def. CG
  * PCG by optimality over K_t(P^-1 A_mu, P^-1 b) Sec. 2.1, def. PCG and
                                                   eq. precond_krylov_def
  * deflation preconditioner and its inverse      Sec. 2.2, eq. precond_def
  * block-Krylov Nystrom approximation A<K_s>     Sec. 2.2.2, eq. nystromBKI_def
  * theta = smallest eigenvalue of the Nystrom
    approximation, same Omega as block-CG          Sec. 7 (numerical experiments)
"""
from __future__ import annotations

import numpy as np

from .block_cg import as_operator, galerkin


def cg_hestenes_stiefel(A, mu, b, t):
    """Textbook conjugate-gradient recurrence (Hestenes-Stiefel) for
    A_mu x = b from x_0 = 0, t steps (t products with A).  In exact
    arithmetic its t-th iterate is cg_t(mu) of def. CG."""
    apply_A = as_operator(A)
    x = np.zeros_like(b, dtype=np.float64)
    r = np.array(b, dtype=np.float64, copy=True)
    p = r.copy()
    rr = r @ r
    for _ in range(t):
        Ap = apply_A(p[:, None])[:, 0] + mu * p
        alpha = rr / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = r @ r
        if rr_new == 0.0:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def krylov_basis_reorth(apply_M, v, t):
    """Orthonormal basis of K_t(M, v) = span{v, Mv, ..., M^(t-1) v} built by
    Arnoldi with two Gram-Schmidt passes; stops early on an invariant space."""
    q = v / np.linalg.norm(v)
    Q = [q]
    for _ in range(t - 1):
        w = apply_M(Q[-1])
        Qm = np.column_stack(Q)
        for _ in range(2):
            w = w - Qm @ (Qm.T @ w)
        nw = np.linalg.norm(w)
        if nw <= 1e-14 * max(1.0, np.linalg.norm(apply_M(Q[-1]))):
            break
        Q.append(w / nw)
    return np.column_stack(Q)


def cg_definition(A, mu, b, t):
    """cg_t(mu) from def. CG: Galerkin solution over K_t(A_mu, b)."""
    apply_A = as_operator(A)
    V = krylov_basis_reorth(lambda v: apply_A(v[:, None])[:, 0] + mu * v, b, t)
    return galerkin(apply_A, mu, V, b)


def nystrom(A, Omega, s):
    """Block-Krylov Nystrom approximation A<K_s> = (A K)(K^T A K)^+ (K^T A)
    with K_s = [Omega, A Omega, ..., A^(s-1) Omega] (eq. nystromBKI_def).

    A<K> depends only on range(K), so an orthonormal basis Q of K_s is used
    instead of the monomial basis; Y = A Q is the s-th pass.  The
    pseudo-inverse is taken through an eigendecomposition of C = Q^T A Q
    with a relative cutoff.  Returns (U, D) with A<K_s> = U diag(D) U^T,
    U orthonormal and D > 0 decreasing."""
    apply_A = as_operator(A)
    Om = np.asarray(Omega, dtype=np.float64)
    blocks = [Om.T]
    for _ in range(s - 1):
        blocks.append(apply_A(blocks[-1]))
    K = np.hstack(blocks)
    Q, _ = np.linalg.qr(K)
    Y = apply_A(Q)
    C = Q.T @ Y
    C = 0.5 * (C + C.T)
    w, V = np.linalg.eigh(C)
    keep = w > 1e-13 * w.max()
    F = Y @ (V[:, keep] / np.sqrt(w[keep]))          # A<K> = F F^T
    U, sig, _ = np.linalg.svd(F, full_matrices=False)
    D = sig ** 2
    keep = D > 1e-13 * D.max()
    return U[:, keep], D[keep]


def nystrom_matrix(U, D):
    return (U * D) @ U.T


def deflation_pinv(U, D, theta, mu):
    """P_mu^-1 = (theta + mu) U (D + mu I)^-1 U^T + (I - U U^T)
    (inverse of eq. precond_def), as a dense matrix."""
    d = U.shape[0]
    return (theta + mu) * (U / (D + mu)) @ U.T + (np.eye(d) - U @ U.T)


def pcg_definition(A, mu, b, Pinv, t):
    """pcg_t(mu) from def. PCG: Galerkin solution in the A_mu-norm over
    K_t(A_mu, b; P_mu) = K_t(P^-1 A_mu, P^-1 b) (eq. precond_krylov_def)."""
    apply_A = as_operator(A)
    M = lambda v: Pinv @ (apply_A(v[:, None])[:, 0] + mu * v)
    V = krylov_basis_reorth(M, Pinv @ b, t)
    return galerkin(apply_A, mu, V, b)


def condition_number_preconditioned(A, mu, Pinv):
    """kappa(P^-1/2 A_mu P^-1/2) = ratio of extreme eigenvalues of the
    generalised problem A_mu v = lambda P v (equivalently of P^-1 A_mu)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    w, V = np.linalg.eigh(0.5 * (Pinv + Pinv.T))
    S = (V * np.sqrt(w)) @ V.T                         # P^-1/2
    M = S @ (A + mu * np.eye(d)) @ S
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    return float(ev[-1] / ev[0])
