"""Dense direct references (float64, CPU).  Test infrastructure only.

These certify the iterative oracle: they compute the exact quantities the
paper's methods approximate, A_mu^-1 b (Sec. 1, eq. regularized_ls), the
ridge path (Sec. 1, eq. ridge_regression) and A^(1/2) b (Sec. 1,
eq. sqrt_rational), by textbook dense factorizations.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def solve_dense(A, mu, b):
    """A_mu^-1 b by Cholesky of A + mu I."""
    A = np.asarray(A, dtype=np.float64)
    c = sla.cho_factor(A + mu * np.eye(A.shape[0]), lower=True)
    return sla.cho_solve(c, np.asarray(b, dtype=np.float64))


def solve_eig(A, mus, B):
    """(A + mu I)^-1 B for many mu from one eigendecomposition.
    B has shape (d,) or (d, r); returns shape (len(mus), d[, r])."""
    w, V = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    VB = V.T @ np.asarray(B, dtype=np.float64)
    return np.stack([V @ (VB / ((w + mu)[:, None] if VB.ndim == 2 else (w + mu))) for mu in mus])


def sqrt_eig(A, B):
    """A^(1/2) B by eigendecomposition; B has shape (m, d), result (m, d)."""
    w, V = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    w = np.maximum(w, 0.0)
    return ((V * np.sqrt(w)) @ (V.T @ np.asarray(B, dtype=np.float64).T)).T


def inv_sqrt_eig(A, B):
    """A^(-1/2) B by eigendecomposition; B has shape (m, d)."""
    w, V = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    return ((V / np.sqrt(w)) @ (V.T @ np.asarray(B, dtype=np.float64).T)).T


def ridge_path_svd(Z, f, mus):
    """Ridge solutions x_mu = argmin ||Z x - f||^2 + mu ||x||^2 for every mu
    via the thin SVD Z = U S V^T: x_mu = V diag(s / (s^2 + mu)) U^T f.
    Avoids forming Z^T Z."""
    Z = np.asarray(Z, dtype=np.float64)
    U, s, Vt = np.linalg.svd(Z, full_matrices=False)
    Uf = U.T @ np.asarray(f, dtype=np.float64)
    return np.stack([Vt.T @ (s / (s * s + mu) * Uf) for mu in mus])


def ridge_path_qr_svd(Z, f, mus, rows_per_block=None, progress=None):
    """Same path through a thin QR of Z (Householder, FP64) and the SVD of the
    triangular factor: Z = Q R, R = U S V^T, x_mu = V diag(s/(s^2+mu)) U^T Q^T f.

    The QR is taken block-row by block-row (tall-skinny QR): Z_i = Q_i R_i,
    then [R_1; ...; R_p] = Q' R, so Q = diag(Q_i) Q' and
    Q^T f = Q'^T [Q_1^T f_1; ...; Q_p^T f_p].  ``progress(i, p)`` is called
    after each block."""
    Z = np.asarray(Z)
    f = np.asarray(f, dtype=np.float64)
    n, d = Z.shape
    rb = rows_per_block or max(d, n)
    Rs, cs = [], []
    nblk = (n + rb - 1) // rb
    for i, r0 in enumerate(range(0, n, rb)):
        Zi = np.asarray(Z[r0:r0 + rb], dtype=np.float64)
        Qi, Ri = np.linalg.qr(Zi, mode="reduced")
        Rs.append(Ri)
        cs.append(Qi.T @ f[r0:r0 + rb])
        del Qi, Zi
        if progress:
            progress(i + 1, nblk)
    if len(Rs) == 1:
        Rf, Qf = Rs[0], cs[0]
    else:
        Q2, Rf = np.linalg.qr(np.vstack(Rs), mode="reduced")
        Qf = Q2.T @ np.concatenate(cs)
    U, s, Vt = np.linalg.svd(Rf)
    Uf = U.T @ Qf
    return np.stack([Vt.T @ (s / (s * s + mu) * Uf) for mu in mus])


def ridge_path_eig_gram(Z, b, mus):
    """Same path from b = Z^T f through the eigendecomposition of Z^T Z
    (right singular vectors / squared singular values of Z)."""
    Z = np.asarray(Z, dtype=np.float64)
    _, s, Vt = np.linalg.svd(Z, full_matrices=False)
    Vb = Vt @ np.asarray(b, dtype=np.float64)
    return np.stack([Vt.T @ (Vb / (s * s + mu)) for mu in mus])
